// Sweep, moments, initialisation, population I/O and exchange kernels for
// populations stored as _Float16 deviations.
#define WLB_STORAGE _Float16
#define WLB_SUFFIX f16
#include "sweep_impl.hpp"
