// Sweep and exchange kernels of the write-coverage check: every population
// store adds one to a 4-byte counter in the population's place (the FP32
// layout), every exchange adds the ghost's counter to its target.
#define WLB_STORAGE cover_t
#define WLB_SUFFIX cover
#include "sweep_impl.hpp"
