// Sweep, moments, initialisation, population I/O and exchange kernels for
// populations stored as bf16_t deviations.
#define WLB_STORAGE bf16_t
#define WLB_SUFFIX bf16
#include "sweep_impl.hpp"
