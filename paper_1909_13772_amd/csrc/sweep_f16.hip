// Sweep, moments, initialisation, population I/O and exchange kernels for
// populations stored as _Float16 deviations.
// At least 6 wavefronts per SIMD for the sweeps (at most 80 VGPRs): the
// 16-bit sweeps are bound by vector instructions and latency, and the extra
// wavefront hides more of it (measured on the 256^3 channel: FP16 48.9k ->
// 51.3k MLUPS, BF16 49.2k -> 50.6k; the odd sweep spills 16 bytes).
#define WLB_WAVES_PER_EU 6
#define WLB_STORAGE _Float16
#define WLB_SUFFIX f16
#include "sweep_impl.hpp"
