// wlb_internal.hpp -- data structures shared by the host runtime and the HIP
// kernels of libwlb.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wlb.h"

namespace wlb {

constexpr int kMaxQ = 27;
constexpr int kWG = 256;  // threads per workgroup of every sweep kernel

// Storage of one block in the arena.  Blocks that follow each other along x
// with the same y-z extent (an x-run) share their rows: row (y, z) holds the
// run's blocks side by side, and each block's xoff is its place in the row.
// Every population slot i is an array
// s_i[z][y][x] over the block's cells, x fastest, with one ghost plane on
// each z side, one ghost row on each y side when the block exchanges along y
// (gy = 1; a block with walls on both y faces has none), and x ghost cells
// only where rows need them.  Rows of 256 bytes or more start interior
// x = 0 on a 128-byte boundary (the alignment rule of the paper's Field,
// Sec. 4.2); a block that wraps onto itself along x has no x ghosts at all
// (xoff 0, rows back to back when the row length is a multiple of 128
// bytes); shorter rows are packed with only their ghost cells (xoff 1):
//   element(i, x, y, z) = pop + i * slot + (z + 1) * plane + (y + gy) * pitch + xoff + x
// for z in [-1, n2], y in [-gy, n1 - 1 + gy].  Besides one descriptor per
// block (used by the ghost exchange), each x-run has a descriptor of its own
// that describes the run as one block (row length W = sum of its blocks' n0,
// the run's x ends and mask); the sweeps and every other tile-based kernel
// work on those, so a tile covers whole stretches of domain rows.  A block's
// mask is its part of the run's mask.  Read with scalar loads.
struct DevBlock {
    int64_t pop;    // element index of slot 0, ghost-inclusive origin (row start of y=-1,z=-1)
    int64_t slot;   // elements per population slot
    int64_t mask;   // index of interior cell (0,0,0) in the u32 mask array; -1 = block has no solid
    int32_t pitch;  // elements per row
    int32_t plane;  // elements per z-plane = pitch * (n1 + 2)
    int32_t n[3];   // interior extent
    int32_t g[3];   // global coordinates of interior cell (0,0,0)
    int32_t mpitch; // mask elements per row (interior only)
    int32_t mplane; // mask elements per plane
    int32_t xoff;   // element offset of interior x = 0 within a row
    int32_t wrapx;  // n[0] if the block is its own neighbour along x (periodic), else 0
    int32_t nbx[2]; // other block across the -x / +x face outside the block's x-run, else -1
    int32_t gy;     // 1: ghost rows on the y faces (the block exchanges along y), 0: none
    int32_t wraplo; // elements added to an access one cell below x = 0 (the run wraps), else 0
    int32_t wraphi; // elements subtracted from an access one cell above x = n0 - 1, else 0
    int32_t pad_;
};
static_assert(sizeof(DevBlock) == 96, "DevBlock layout");

// One tile of a sweep: block id and start/extent (extent <= 256 cells).
// Packed as int4 {block, x0 | ex << 16, y0 | ey << 16, z0 | ez << 16}.  A
// list tile (sweeps only) is {block, first entry in the cell list, 0, -count}
// with up to 256 fluid cells of the block.
struct TileHost {
    int32_t b, x0, y0, z0, ex, ey, ez;
};

// Exchange work item: copy population `slot` over a rectangular region of
// cells from block sb (coordinates s0 + r) to block db (coordinates d0 + r),
// r over the linear cell range [start, start + count) of a region with
// extents (ex, ey, *), count <= kXChunk.  chk >= 0: skip cells whose
// destination mask has bit chk or the solid bit set (used after the odd
// sweep).
constexpr int kXChunk = 4 * kWG;
struct XItem {
    int32_t sb, db;
    int32_t slot, chk;
    int32_t ex, ey;
    int32_t s0[3];
    int32_t d0[3];
    int32_t start, count;
};
static_assert(sizeof(XItem) == 56, "XItem layout");

// Mask word of a cell: bit i (i < 27) set when the neighbour x + c_i is a
// solid cell; bit 31 set when the cell itself is solid.
constexpr uint32_t kSolidBit = 0x80000000u;

// Runtime parameters of a sweep (uniform, passed by value).
struct SweepArgs {
    void *arena;
    const DevBlock *blocks;
    const int4 *tiles;      // box tiles (every kernel but the sweeps)
    const int4 *stiles;     // tiles of the sweeps: the box tiles, or lists of fluid cells
    const uint32_t *cells;  // packed fluid cells x | y << 10 | z << 20 of the list tiles
    const uint32_t *masks;
    const void *mlp;  // MlpDev of the learned closure (closure == 2)
    int32_t ntiles;
    int32_t nstiles;
    int32_t dom[3];
    int32_t periodic;      // bit a set: axis a wraps
    int32_t pressure_axis; // -1 or axis
    int32_t closure;
    int32_t lds_stride;    // > 0: odd sweep stages x-shifted populations in LDS rows of this many elements
    int32_t lds_ring;      // 1: every tile is a whole row of a self-wrapping block (staged sweep without halos)
    int32_t xcd_map;       // 1: one workgroup per tile, each XCD takes a contiguous range of tiles
    int32_t nt;            // 1: the sweep's population accesses carry the non-temporal hint; 2 (odd
                           // sweep): only its aligned ones (populations with c_x = 0)
    int32_t vec_odd;       // 1: the odd sweep moves whole rows as 16-byte vectors per lane (vtiles)
    int32_t nvtiles;
    const int4 *vtiles;    // row tiles of the vector odd sweep: {block, 0 | n0 << 16, y0 | ey << 16, z0 | ez << 16}
    double omega;          // 1 / tau0
    double omega_minus;    // TRT rate of the antisymmetric part at tau0
    double magic;          // TRT Lambda
    double omega_bulk;
    double omega_higher;
    double force[3];
    double rho_in, rho_out;
    double tau0;
    double smag_k;         // 18 sqrt(2) C_s^2
};

// Arguments of the moments / reduction pass.
struct MomArgs {
    SweepArgs s;
    int32_t swapped;       // 1: layout after an even sweep (read like the odd sweep)
    int32_t z0, z1;        // global z range written to out (out == nullptr: none)
    double *out;           // [4][ncells of slab]: rho, ux, uy, uz in global order of the slab
    double *partials;      // [ntiles][8] or nullptr
};

// Kernel launchers, one set per storage type (sweep_<type>.hip).
#define WLB_DECLARE_LAUNCHERS(S)                                                                              \
    hipError_t sweep_##S(int q, int coll, bool odd, const SweepArgs &a, int grid, hipStream_t st);            \
    hipError_t moments_##S(int q, const MomArgs &a, int grid, hipStream_t st);                               \
    hipError_t force_##S(int q, const SweepArgs &a, double *partials, int grid, hipStream_t st);              \
    hipError_t init_##S(int q, const SweepArgs &a, const double *rhou, int z0, int z1, int grid,             \
                        hipStream_t st);                                                                      \
    hipError_t pdfs_##S(int q, const SweepArgs &a, double *buf, int z0, int z1, bool to_device, bool swapped, \
                        int grid, hipStream_t st);                                                            \
    hipError_t exchange_##S(void *arena, const DevBlock *blocks, const uint32_t *masks, const XItem *items,   \
                            int nitems, int xcd_map, hipStream_t st);                                         \
    hipError_t filter_##S(int q, const SweepArgs &a, int fac, double *out, int64_t ncoarse, bool swapped,       \
                          hipStream_t st);
WLB_DECLARE_LAUNCHERS(f64)
WLB_DECLARE_LAUNCHERS(f32)
WLB_DECLARE_LAUNCHERS(f16)
WLB_DECLARE_LAUNCHERS(bf16)
WLB_DECLARE_LAUNCHERS(cover)  // write-coverage check (4-byte counters in the FP32 layout)

// Learned closure (mlp_train.hip).
hipError_t launch_mlp_forward(const void *net, const float *raw, int64_t n, float *out, int32_t *flag, hipStream_t st);
size_t mlp_grad_workspace_bytes(int64_t n);
// largest minibatch of the gradient pass without a caller workspace, and the
// device address of this GPU's copy of its partial-sum array
constexpr int64_t kMlpNoAllocMaxSamples = WLB_MLP_NOALLOC_MAX_SAMPLES;
constexpr int kMaxDevices = 64;
hipError_t mlp_scratch_address(void **out);
hipError_t launch_mlp_grad(const float *P, const float *raw, const float *target, int64_t n, float inv_scale,
                           float *grad, float *loss, float *work, hipStream_t st);
hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t st);
// Builds the per-lane device layout of the network from packed float params.
void mlp_prepare(const float *params, void *mlpdev_host);
size_t mlp_dev_bytes();

// Storage-independent kernels (misc.hip).
hipError_t launch_masks(const SweepArgs &a, const uint8_t *solid, int q, int grid, hipStream_t st);
hipError_t launch_reduce_totals(const double *partials, int n, double *out8, hipStream_t st);
hipError_t launch_reduce_sum8(const double *partials, int n, double *out8, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);
hipError_t launch_les_targets(const double *filt, const int32_t nc[3], double tau0, float *raw, float *target,
                              hipStream_t st);

}  // namespace wlb
