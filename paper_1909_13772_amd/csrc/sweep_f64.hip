// Sweep, moments, initialisation, population I/O and exchange kernels for
// populations stored as double deviations.
#define WLB_STORAGE double
#define WLB_SUFFIX f64
#include "sweep_impl.hpp"
