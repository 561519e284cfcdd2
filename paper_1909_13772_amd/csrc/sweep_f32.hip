// Sweep, moments, initialisation, population I/O and exchange kernels for
// populations stored as float deviations.
#define WLB_STORAGE float
#define WLB_SUFFIX f32
#include "sweep_impl.hpp"
