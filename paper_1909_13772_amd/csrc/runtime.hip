// runtime.hip -- host runtime and C ABI of libwlb.so.
//
// Blocks (paper Sec. 3.1, Sec. 4.1) become descriptors of one device arena
// that the caller allocates; a time step is a sweep over all blocks followed
// by a ghost-layer exchange (Sec. 4.2), the exchange between blocks of the
// same device being a direct copy without buffers (Sec. 3.3).  Host arrays
// are copied in at set-up and out after many steps (Sec. 4.3).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wlb.h"
#include "lattice.hpp"
#include "wlb_internal.hpp"

using namespace wlb;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail(WLB_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Tile-shape candidates of the autotuner; (0,0,0) packs whole rows.
const int kShapes[][3] = {{0, 0, 0}, {64, 4, 1}, {32, 8, 1}, {32, 4, 2}, {16, 16, 1}, {16, 4, 4},
                          {128, 2, 1}, {256, 1, 1}, {64, 2, 2}, {8, 8, 4}};
// 0: one workgroup per tile; -1: the same with XCD-contiguous tile ranges;
// > 0: persistent grid of that many workgroups
const int kGrids[] = {0, -1, 1024, 2048, 4096};

struct HostBlock {
    int org[3], n[3];
    int nbr[27];  // neighbour block for offset index (ox+1) + 3 (oy+1) + 9 (oz+1); -1 none
};

}  // namespace

struct wlb_blocks {
    int q = 19, storage = 0, esize = 8;
    int dom[3] = {0, 0, 0}, periodic[3] = {0, 0, 0};
    std::vector<HostBlock> blocks;
    // Blocks that follow each other along x with the same y-z extent form an
    // x-run and share their population rows.  dev[0, n) describes the
    // blocks (exchange, coverage), dev[n + r] run r as one block: every
    // tile-based kernel works on runs, so a tile's rows are whole stretches
    // of a domain row instead of the pieces that fall into one block.
    std::vector<DevBlock> dev;
    int nblk = 0;
    std::vector<std::vector<int>> runs;
    // population slots: run_slot0[r] elements per slot of run r before the
    // stride rounding; slots of 64 MiB or more are rounded up to a multiple
    // of slot_round bytes (an autotuner candidate, see relayout_slots)
    std::vector<int64_t> run_slot0;
    size_t slot_round = (size_t)16 << 20;
    std::vector<HostBlock> rhost;  // extent and y/z neighbour flags of each run
    std::vector<TileHost> tiles;
    std::vector<XItem> pull, push;
    int64_t ncells = 0, nfluid = 0, xchg_elems = 0;
    // arena layout (bytes)
    size_t off_pop = 0, pop_bytes = 0, off_mask = 0, mask_words = 0, off_blocks = 0, off_tiles = 0,
           tile_cap = 0, off_pull = 0, off_push = 0, off_partials = 0, off_totals = 0, off_stage = 0,
           stage_bytes = 0, off_mlp = 0, arena_bytes = 0, off_cells = 0, off_ltiles = 0, ltile_cap = 0,
           off_vtiles = 0, vtile_cap = 0;
    char *arena = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false, inited = false;
    int collision = 0;
    wlb_lbm_params params{};
    std::vector<float> mlp;
    SweepArgs args{};
    int64_t steps = 0;
    int parity = 0;       // 0 natural layout, 1 swapped (after an even sweep)
    int pending = 0;      // 0 none, 1 pull due (after even), 2 push due (after odd)
    // sweep tiles as lists of fluid cells (porous media); available after an
    // init with solid cells when every block fits the 10/10/12-bit packing
    bool list_ok = false, list_built = false, list_mode = false;
    std::vector<int4> ltiles;
    int last_sweep = -1;  // parity of the last sweep (-1: none since init / set)
    int shape[3] = {0, 0, 0};
    // per-run tile shape set by the autotuner for classes of runs (runs of
    // one y extent); empty: `shape` for every run
    std::vector<std::array<int, 3>> run_shape;
    int grid = 0;
    bool lds_stage = false;  // odd sweep stages x-shifted populations in LDS (autotuner candidate)
    // odd sweep over whole rows with 16-byte vectors per lane (autotuner
    // candidate); possible when every block wraps onto itself along x, has
    // no solid cells nearby and rows split into whole vectors
    bool vec_want = false, vec_ok = false;
    std::vector<int4> vtiles;
    // interior/frontier overlap: each sweep is split into the cells at least
    // kFrontier rows away from every y/z face with a neighbour (interior) and
    // the rest (frontier); the frontier and the exchange run on a second
    // stream while the interior runs on the bound stream (autotuner candidate)
    bool overlap = false;
    bool cover = false;   // sweeps and exchanges count writes (wlb_debug_write_coverage)
    // non-temporal population accesses per parity (autotuner candidates); the
    // odd sweep: 0 none, 1 every access, 2 its aligned accesses only
    bool nt_even = true;
    int nt_odd = 1;
    int nint_tiles = 0;   // interior box tiles come first in `tiles` when split
    int nint_ltiles = 0;  // interior fluid-cell tiles come first in `ltiles`
    bool tiles_split = false;
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool use_graph = true;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool graph_valid = false;
    // kernel timing
    bool timing = false;
    struct Ev {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Ev> ev_pool;
    size_t ev_used = 0;
    double ms[4] = {0, 0, 0, 0};
    int64_t cnt[4] = {0, 0, 0, 0};
};

namespace {

int storage_esize(int s) { return s == WLB_F64 ? 8 : (s == WLB_F32 ? 4 : 2); }

// Rows at most this far from a y/z face with a neighbour block form the
// frontier: the exchange reads and writes the row at the face and its ghost
// row, and the odd sweep of the next row in touches the row at the face.
constexpr int kFrontier = 2;

// Interior rectangle (y0, y1) x (z0, z1) of block B: rows of every cell that
// neither reads a ghost row nor touches the row at a face with a neighbour.
// Empty when the block is too thin.
void interior_rows(const HostBlock &B, int &y0, int &y1, int &z0, int &z1)
{
    y0 = B.nbr[10] >= 0 ? kFrontier : 0;  // neighbour at -y
    y1 = B.n[1] - (B.nbr[16] >= 0 ? kFrontier : 0);
    z0 = B.nbr[4] >= 0 ? kFrontier : 0;
    z1 = B.n[2] - (B.nbr[22] >= 0 ? kFrontier : 0);
    if (y0 >= y1 || z0 >= z1) y0 = y1 = z0 = z1 = 0;
}

bool in_interior(int y, int z, int y0, int y1, int z0, int z1) { return y >= y0 && y < y1 && z >= z0 && z < z1; }

// Box tiles of block b over rows [y0, y1) x [z0, z1) (all x).  tx = 0 packs
// whole rows.
void tile_region(const HostBlock &B, int b, int tx, int ty, int tz, int y0, int y1, int z0, int z1,
                 std::vector<TileHost> &out)
{
    if (y0 >= y1 || z0 >= z1) return;
    int ex, ey, ez;
    if (tx == 0) {
        ex = std::min(B.n[0], kWG);
        ey = std::min(y1 - y0, std::max(1, kWG / ex));
        ez = std::min(z1 - z0, std::max(1, kWG / (ex * ey)));
    } else {
        ex = std::min(tx, B.n[0]);
        ey = std::min(ty, y1 - y0);
        ez = std::min(tz, z1 - z0);
    }
    for (int z = z0; z < z1; z += ez)
        for (int y = y0; y < y1; y += ey)
            for (int x = 0; x < B.n[0]; x += ex) {
                TileHost t;
                t.b = b;
                t.x0 = x;
                t.y0 = y;
                t.z0 = z;
                t.ex = std::min(ex, B.n[0] - x);
                t.ey = std::min(ey, y1 - y);
                t.ez = std::min(ez, z1 - z);
                out.push_back(t);
            }
}

// Largest slot stride rounding the autotuner tries: the arena is sized for it.
constexpr size_t kSlotRoundMax = (size_t)16 << 20;

// Places the population slots of every x-run one after the other.  The
// sweeps stream all q slots at the same cell offset at once, and on MI355X
// the achieved bandwidth of that access pattern depends on the slots'
// stride, not monotonically (stand-alone even pattern over a 256^3 FP64
// block: 0.82 ms at a 128 MiB stride, 0.96 ms at 129 MiB, 0.83 ms at 130
// MiB and at 144 MiB).  Slots of 64 MiB or more are therefore rounded up to
// a multiple of `round` bytes (0: alignment only), which the autotuner
// chooses by measurement; smaller slots are only aligned.  Sets pop and
// slot of every block and run descriptor; returns the elements used.
size_t relayout_slots(wlb_blocks *h, size_t round)
{
    size_t elems = 0;
    for (size_t r = 0; r < h->runs.size(); ++r) {
        int64_t slot = h->run_slot0[r];
        if (round && slot * h->esize >= ((int64_t)64 << 20)) slot = (int64_t)(round_up((size_t)slot * h->esize, round) / h->esize);
        const int64_t pop = (int64_t)elems;
        elems += (size_t)slot * h->q;
        for (int m : h->runs[r]) {
            h->dev[m].slot = slot;
            h->dev[m].pop = pop;
        }
        h->dev[h->nblk + r].slot = slot;
        h->dev[h->nblk + r].pop = pop;
    }
    h->slot_round = round;
    return elems;
}

// Sweep tiles of every x-run.  split: interior tiles first (their count in
// *nint), then the frontier, each group in longest-processing-time order
// for the persistent (grid-stride) launch.  Box tiles (tx >= 0) take the
// run's own shape where the autotuner set one (h->run_shape).
void build_tiles(const wlb_blocks *h, int tx, int ty, int tz, std::vector<TileHost> &out, bool split = false,
                 int *nint = nullptr)
{
    out.clear();
    std::vector<TileHost> outer;
    for (int r = 0; r < (int)h->rhost.size(); ++r) {
        const HostBlock &B = h->rhost[r];
        const int b = h->nblk + r;
        int sx = tx, sy = ty, sz = tz;
        if (!h->run_shape.empty() && tx >= 0) {
            sx = h->run_shape[r][0];
            sy = h->run_shape[r][1];
            sz = h->run_shape[r][2];
        }
        if (!split) {
            tile_region(B, b, sx, sy, sz, 0, B.n[1], 0, B.n[2], out);
            continue;
        }
        int y0, y1, z0, z1;
        interior_rows(B, y0, y1, z0, z1);
        tile_region(B, b, sx, sy, sz, y0, y1, z0, z1, out);
        if (y0 >= y1) {  // no interior: the whole run is frontier
            tile_region(B, b, sx, sy, sz, 0, B.n[1], 0, B.n[2], outer);
            continue;
        }
        tile_region(B, b, sx, sy, sz, 0, B.n[1], 0, z0, outer);
        tile_region(B, b, sx, sy, sz, 0, B.n[1], z1, B.n[2], outer);
        tile_region(B, b, sx, sy, sz, 0, y0, z0, z1, outer);
        tile_region(B, b, sx, sy, sz, y1, B.n[1], z0, z1, outer);
    }
    auto lpt = [](const TileHost &a, const TileHost &b) { return a.ex * a.ey * a.ez > b.ex * b.ey * b.ez; };
    std::stable_sort(out.begin(), out.end(), lpt);
    std::stable_sort(outer.begin(), outer.end(), lpt);
    if (nint) *nint = (int)out.size();
    out.insert(out.end(), outer.begin(), outer.end());
}

size_t count_tiles(const wlb_blocks *h, int tx, int ty, int tz, bool split = false)
{
    std::vector<TileHost> t;
    build_tiles(h, tx, ty, tz, t, split);
    return t.size();
}

// Row-buffer length of the LDS-staged odd sweep: the largest tile's rows
// times (segment length + 2 halo cells).  Staging is used only when it fits
// in 64 KiB of LDS per workgroup.
void update_lds_stride(wlb_blocks *h)
{
    int stride = 0;
    bool ring = true;
    for (const TileHost &t : h->tiles) {
        stride = std::max(stride, t.ey * t.ez * (t.ex + 2));
        ring = ring && t.ex == h->dev[t.b].n[0] && h->dev[t.b].wrapx != 0;
    }
    h->args.lds_ring = ring ? 1 : 0;
    int nsh = 0;  // populations with c_x != 0 (the staged ones)
    for (int i = 0; i < h->q; ++i) nsh += ccq(h->q, i, 0) != 0;
    const size_t bytes = (((size_t)nsh * stride * h->esize + 15) & ~(size_t)15) + kWG * 4;
    h->args.lds_stride = (h->lds_stage && bytes <= 65536 && !h->list_mode) ? stride : 0;
    // the row-vector odd sweep takes whole rows of its own tiles; it has no
    // interior / frontier split, so the overlap turns it off
    h->args.vec_odd = (h->vec_want && h->vec_ok && !h->overlap) ? 1 : 0;
    if (h->args.vec_odd) h->args.lds_stride = 0;
    h->graph_valid = false;
}

// Elements per 16-byte vector of the storage type.
int row_vec(const wlb_blocks *h) { return 16 / h->esize; }

// Row tiles of the vector odd sweep (after the masks are known).  A tile is
// floor(256 / (W / V)) rows of one x-run (row length W) along y.
int build_vtiles(wlb_blocks *h)
{
    const int V = row_vec(h);
    h->vec_ok = h->params.closure != WLB_CLOSURE_MLP && !h->rhost.empty();
    for (size_t b = h->nblk; b < h->dev.size() && h->vec_ok; ++b) {
        const DevBlock &D = h->dev[b];
        const int L = D.n[0] / V;
        if (D.wrapx == 0 || D.mask >= 0 || D.xoff != 0 || D.n[0] % V != 0 || L > kWG || L < 1) h->vec_ok = false;
    }
    h->vtiles.clear();
    if (!h->vec_ok) return WLB_OK;
    for (size_t b = h->nblk; b < h->dev.size(); ++b) {
        const DevBlock &D = h->dev[b];
        const int R = kWG / (D.n[0] / V);
        for (int z = 0; z < D.n[2]; ++z)
            for (int y0 = 0; y0 < D.n[1]; y0 += R)
                h->vtiles.push_back(make_int4((int)b, D.n[0] << 16, y0 | (std::min(R, D.n[1] - y0) << 16), z | (1 << 16)));
    }
    if (h->vtiles.size() > h->vtile_cap) {
        h->vtiles.clear();
        h->vec_ok = false;
        return WLB_OK;
    }
    HIPCHK(hipMemcpyAsync(h->arena + h->off_vtiles, h->vtiles.data(), h->vtiles.size() * sizeof(int4),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->args.vtiles = reinterpret_cast<const int4 *>(h->arena + h->off_vtiles);
    h->args.nvtiles = (int)h->vtiles.size();
    return WLB_OK;
}

int upload_tiles(wlb_blocks *h)
{
    std::vector<int4> packed(h->tiles.size());
    for (size_t k = 0; k < h->tiles.size(); ++k) {
        const TileHost &t = h->tiles[k];
        packed[k] = make_int4(t.b, t.x0 | (t.ex << 16), t.y0 | (t.ey << 16), t.z0 | (t.ez << 16));
    }
    HIPCHK(hipMemcpyAsync(h->arena + h->off_tiles, packed.data(), packed.size() * sizeof(int4),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->args.ntiles = (int)h->tiles.size();
    if (h->list_mode) {
        h->args.stiles = reinterpret_cast<const int4 *>(h->arena + h->off_ltiles);
        h->args.nstiles = (int)h->ltiles.size();
    } else {
        h->args.stiles = h->args.tiles;
        h->args.nstiles = h->args.ntiles;
    }
    update_lds_stride(h);
    return WLB_OK;
}

int set_tiles(wlb_blocks *h, int tx, int ty, int tz, int grid)
{
    // tx = -1: sweeps over lists of fluid cells, whole-row boxes elsewhere
    const bool list = tx == -1;
    if (list && !h->list_built) return fail(WLB_ERR_STATE, "fluid-cell tiles need an init with solid cells");
    std::vector<TileHost> t;
    int nint = 0;
    build_tiles(h, list ? 0 : tx, ty, tz, t, h->overlap, &nint);
    if (t.size() > h->tile_cap) return fail(WLB_ERR_ARG, "tile shape yields %zu tiles > capacity", t.size());
    h->tiles.swap(t);
    h->nint_tiles = nint;
    h->tiles_split = h->overlap;
    h->shape[0] = tx;
    h->shape[1] = ty;
    h->shape[2] = tz;
    h->grid = grid;
    h->list_mode = list;
    h->args.xcd_map = grid == -1 ? 1 : 0;
    h->graph_valid = false;
    if (h->bound) return upload_tiles(h);
    return WLB_OK;
}

int launch_grid(const wlb_blocks *h)
{
    const int n = (int)(h->list_mode ? h->ltiles.size() : h->tiles.size());
    if (h->grid <= 0 || h->grid > n) return n > 0 ? n : 1;
    return h->grid;
}

hipError_t sweep_launch(const wlb_blocks *h, bool odd, const SweepArgs &args, int g, hipStream_t st)
{
    SweepArgs a = args;
    a.nt = odd ? h->nt_odd : (h->nt_even ? 1 : 0);
    // the row-vector odd sweep exists for FP64 storage (and the counting
    // storage of the write-coverage check); other storage runs the direct one
    if (a.vec_odd && !(h->esize == 8 || h->cover)) a.vec_odd = 0;
    if (odd && a.vec_odd) g = (h->grid > 0 && h->grid < a.nvtiles) ? h->grid : std::max(1, a.nvtiles);
    if (h->cover) return sweep_cover(h->q, h->collision, odd, a, g, st);
    switch (h->storage) {
    case WLB_F64: return sweep_f64(h->q, h->collision, odd, a, g, st);
    case WLB_F32: return sweep_f32(h->q, h->collision, odd, a, g, st);
    case WLB_F16DEV: return sweep_f16(h->q, h->collision, odd, a, g, st);
    default: return sweep_bf16(h->q, h->collision, odd, a, g, st);
    }
}

// The sweep is launched as an interior and a frontier part.
bool split_sweeps(const wlb_blocks *h) { return h->overlap && (h->list_mode || h->tiles_split); }

// Arguments of one part of a split sweep (its tiles and their count in *n)
// and its workgroup count.
SweepArgs part_args(const wlb_blocks *h, bool interior, int *n, int *grid)
{
    SweepArgs a = h->args;
    const int nint = h->list_mode ? h->nint_ltiles : h->nint_tiles;
    if (interior) {
        a.nstiles = nint;
    } else {
        a.stiles = a.stiles + nint;
        a.nstiles = a.nstiles - nint;
    }
    *n = a.nstiles;
    *grid = (h->grid <= 0 || h->grid > *n) ? *n : h->grid;
    return a;
}

// Whole sweep on the bound stream (both parts in turn when split).
hipError_t sweep_dispatch(const wlb_blocks *h, bool odd)
{
    if (!split_sweeps(h)) return sweep_launch(h, odd, h->args, launch_grid(h), h->stream);
    for (int part = 0; part < 2; ++part) {
        int n = 0, g = 0;
        const SweepArgs a = part_args(h, part == 0, &n, &g);
        if (n > 0) {
            const hipError_t e = sweep_launch(h, odd, a, g, h->stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t exchange_dispatch(const wlb_blocks *h, bool after_odd, hipStream_t st = nullptr)
{
    if (!st) st = h->stream;
    const std::vector<XItem> &v = after_odd ? h->push : h->pull;
    const XItem *items = reinterpret_cast<const XItem *>(h->arena + (after_odd ? h->off_push : h->off_pull));
    const DevBlock *blocks = reinterpret_cast<const DevBlock *>(h->arena + h->off_blocks);
    const uint32_t *masks = reinterpret_cast<const uint32_t *>(h->arena + h->off_mask);
    void *pops = h->arena + h->off_pop;
    const int n = (int)v.size();
    const int xm = h->args.xcd_map;
    if (h->cover) return exchange_cover(pops, blocks, masks, items, n, xm, st);
    switch (h->storage) {
    case WLB_F64: return exchange_f64(pops, blocks, masks, items, n, xm, st);
    case WLB_F32: return exchange_f32(pops, blocks, masks, items, n, xm, st);
    case WLB_F16DEV: return exchange_f16(pops, blocks, masks, items, n, xm, st);
    default: return exchange_bf16(pops, blocks, masks, items, n, xm, st);
    }
}

hipError_t moments_dispatch(const wlb_blocks *h, const MomArgs &m, int grid)
{
    switch (h->storage) {
    case WLB_F64: return moments_f64(h->q, m, grid, h->stream);
    case WLB_F32: return moments_f32(h->q, m, grid, h->stream);
    case WLB_F16DEV: return moments_f16(h->q, m, grid, h->stream);
    default: return moments_bf16(h->q, m, grid, h->stream);
    }
}

hipError_t force_dispatch(const wlb_blocks *h, double *partials, int grid)
{
    switch (h->storage) {
    case WLB_F64: return force_f64(h->q, h->args, partials, grid, h->stream);
    case WLB_F32: return force_f32(h->q, h->args, partials, grid, h->stream);
    case WLB_F16DEV: return force_f16(h->q, h->args, partials, grid, h->stream);
    default: return force_bf16(h->q, h->args, partials, grid, h->stream);
    }
}

hipError_t init_dispatch(const wlb_blocks *h, const double *rhou, int z0, int z1, int grid)
{
    switch (h->storage) {
    case WLB_F64: return init_f64(h->q, h->args, rhou, z0, z1, grid, h->stream);
    case WLB_F32: return init_f32(h->q, h->args, rhou, z0, z1, grid, h->stream);
    case WLB_F16DEV: return init_f16(h->q, h->args, rhou, z0, z1, grid, h->stream);
    default: return init_bf16(h->q, h->args, rhou, z0, z1, grid, h->stream);
    }
}

hipError_t pdfs_dispatch(const wlb_blocks *h, double *buf, int z0, int z1, bool to_dev, bool swapped, int grid)
{
    switch (h->storage) {
    case WLB_F64: return pdfs_f64(h->q, h->args, buf, z0, z1, to_dev, swapped, grid, h->stream);
    case WLB_F32: return pdfs_f32(h->q, h->args, buf, z0, z1, to_dev, swapped, grid, h->stream);
    case WLB_F16DEV: return pdfs_f16(h->q, h->args, buf, z0, z1, to_dev, swapped, grid, h->stream);
    default: return pdfs_bf16(h->q, h->args, buf, z0, z1, to_dev, swapped, grid, h->stream);
    }
}

// Grid for the auxiliary (non-hot) passes.
int aux_grid(const wlb_blocks *h)
{
    const int n = (int)h->tiles.size();
    return n < 8192 ? (n > 0 ? n : 1) : 8192;
}

// --- kernel timing -------------------------------------------------------
int fold_events(wlb_blocks *h)
{
    if (h->ev_used == 0) return WLB_OK;
    HIPCHK(hipEventSynchronize(h->ev_pool[h->ev_used - 1].b));
    for (size_t k = 0; k < h->ev_used; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev_pool[k].a, h->ev_pool[k].b));
        h->ms[h->ev_pool[k].kind] += ms;
        h->cnt[h->ev_pool[k].kind] += 1;
    }
    h->ev_used = 0;
    return WLB_OK;
}

int timed_begin(wlb_blocks *h, int kind, size_t *slot)
{
    if (h->ev_used == h->ev_pool.size()) {
        if (h->ev_pool.size() >= 4096) {
            int rc = fold_events(h);
            if (rc) return rc;
        } else {
            wlb_blocks::Ev e;
            HIPCHK(hipEventCreate(&e.a));
            HIPCHK(hipEventCreate(&e.b));
            h->ev_pool.push_back(e);
        }
    }
    *slot = h->ev_used++;
    h->ev_pool[*slot].kind = kind;
    HIPCHK(hipEventRecord(h->ev_pool[*slot].a, h->stream));
    return WLB_OK;
}

int run_sweep(wlb_blocks *h, bool odd)
{
    size_t s = 0;
    if (h->timing) {
        int rc = timed_begin(h, odd ? 1 : 0, &s);
        if (rc) return rc;
    }
    HIPCHK(sweep_dispatch(h, odd));
    if (h->timing) HIPCHK(hipEventRecord(h->ev_pool[s].b, h->stream));
    return WLB_OK;
}

int run_exchange(wlb_blocks *h, bool after_odd)
{
    size_t s = 0;
    if (h->timing) {
        int rc = timed_begin(h, after_odd ? 3 : 2, &s);
        if (rc) return rc;
    }
    HIPCHK(exchange_dispatch(h, after_odd));
    if (h->timing) HIPCHK(hipEventRecord(h->ev_pool[s].b, h->stream));
    return WLB_OK;
}

// Second stream and the fork / join events of the overlap (default
// priority, like the bound stream).
int ensure_stream2(wlb_blocks *h)
{
    if (!h->stream2) HIPCHK(hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
    if (!h->ev_fork) HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    if (!h->ev_join) HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    return WLB_OK;
}

// One step (sweep of the current parity, then its exchange).  With the
// overlap, the frontier part of the sweep and the exchange run on the second
// stream while the interior part runs on the bound stream; the step ends
// when both have finished.  The exchange reads and writes only rows at block
// faces and ghost rows, which no interior cell touches, and every population
// location of a sweep belongs to exactly one cell, so the parts need no other
// ordering.
int enqueue_step(wlb_blocks *h, bool odd)
{
    if (!split_sweeps(h) || !h->stream2) {
        HIPCHK(sweep_dispatch(h, odd));
        HIPCHK(exchange_dispatch(h, odd));
        return WLB_OK;
    }
    HIPCHK(hipEventRecord(h->ev_fork, h->stream));
    HIPCHK(hipStreamWaitEvent(h->stream2, h->ev_fork, 0));
    int n = 0, g = 0;
    const SweepArgs af = part_args(h, false, &n, &g);
    if (n > 0) HIPCHK(sweep_launch(h, odd, af, g, h->stream2));
    HIPCHK(exchange_dispatch(h, odd, h->stream2));
    const SweepArgs ai = part_args(h, true, &n, &g);
    if (n > 0) HIPCHK(sweep_launch(h, odd, ai, g, h->stream));
    HIPCHK(hipEventRecord(h->ev_join, h->stream2));
    HIPCHK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    return WLB_OK;
}

int one_step(wlb_blocks *h)
{
    const bool odd = h->parity == 1;
    int rc;
    if (h->timing) {  // per-kernel events: the parts run in turn on the bound stream
        rc = run_sweep(h, odd);
        if (rc) return rc;
        rc = run_exchange(h, odd);
    } else {
        rc = enqueue_step(h, odd);
    }
    if (rc) return rc;
    h->parity ^= 1;
    h->pending = 0;
    h->last_sweep = odd ? 1 : 0;
    h->steps += 1;
    return WLB_OK;
}

void drop_graph(wlb_blocks *h)
{
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    if (h->graph) hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    h->graph_valid = false;
}

int capture_graph(wlb_blocks *h)
{
    drop_graph(h);
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const int r1 = enqueue_step(h, false);
    const int r2 = r1 ? r1 : enqueue_step(h, true);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(h->stream, &g);
    if (r1 || r2 || ec != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail(WLB_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ec != hipSuccess ? ec : hipErrorUnknown));
    }
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    h->graph_valid = true;
    return WLB_OK;
}

// Deterministic FP64 totals of the current state into arena totals slot;
// copies them to `host8` when non-null (synchronises).
int compute_totals(wlb_blocks *h, double *host8)
{
    MomArgs m{};
    m.s = h->args;
    m.swapped = h->parity;
    m.z0 = 0;
    m.z1 = 0;
    m.out = nullptr;
    m.partials = reinterpret_cast<double *>(h->arena + h->off_partials);
    HIPCHK(moments_dispatch(h, m, aux_grid(h)));
    double *tot = reinterpret_cast<double *>(h->arena + h->off_totals);
    HIPCHK(launch_reduce_totals(m.partials, (int)h->tiles.size(), tot, h->stream));
    if (host8) {
        HIPCHK(hipMemcpyAsync(host8, tot, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        host8[7] = (double)h->steps;
    }
    return WLB_OK;
}

int health_check(wlb_blocks *h)
{
    double t[8];
    int rc = compute_totals(h, t);
    if (rc) return rc;
    const double lim = h->params.health_umax > 0 ? h->params.health_umax : 0.3;
    if (!std::isfinite(t[0]) || !std::isfinite(t[5]) || t[5] > lim)
        return fail(WLB_ERR_DIVERGED, "health check failed at step %lld: mass %g, max|u| %g",
                    (long long)h->steps, t[0], t[5]);
    return WLB_OK;
}

int planes_per_chunk(const wlb_blocks *h, size_t bytes_per_cell)
{
    const size_t plane = (size_t)h->dom[0] * h->dom[1] * bytes_per_cell;
    size_t k = h->stage_bytes / plane;
    if (k < 1) k = 1;
    if (k > (size_t)h->dom[2]) k = h->dom[2];
    return (int)k;
}

int do_init_state(wlb_blocks *h, const double *rho, const double *u)
{
    const int64_t plane = (int64_t)h->dom[0] * h->dom[1];
    const int64_t N = plane * h->dom[2];
    const int kz = planes_per_chunk(h, 4 * sizeof(double));
    double *stage = reinterpret_cast<double *>(h->arena + h->off_stage);
    for (int z0 = 0; z0 < h->dom[2]; z0 += kz) {
        const int z1 = std::min(h->dom[2], z0 + kz);
        const int64_t S = (int64_t)(z1 - z0) * plane;
        HIPCHK(hipMemcpyAsync(stage, rho + z0 * plane, S * sizeof(double), hipMemcpyHostToDevice, h->stream));
        for (int a = 0; a < 3; ++a)
            HIPCHK(hipMemcpyAsync(stage + (1 + a) * S, u + a * N + z0 * plane, S * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream));
        HIPCHK(init_dispatch(h, stage, z0, z1, aux_grid(h)));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->steps = 0;
    h->parity = 0;
    h->pending = 0;
    h->last_sweep = -1;
    return WLB_OK;
}

int time_pairs(wlb_blocks *h, int reps, float *ms_out)
{
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    // warm-up pair
    for (int k = 0; k < 2; ++k) {
        int rc = enqueue_step(h, false);
        if (!rc) rc = enqueue_step(h, true);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(a, h->stream));
    for (int k = 0; k < reps; ++k) {
        int rc = enqueue_step(h, false);
        if (!rc) rc = enqueue_step(h, true);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(b, h->stream));
    HIPCHK(hipEventSynchronize(b));
    HIPCHK(hipEventElapsedTime(ms_out, a, b));
    *ms_out /= reps;
    hipEventDestroy(a);
    hipEventDestroy(b);
    return WLB_OK;
}

// Factor by which a candidate must beat the best time so far to replace it.
constexpr float kTuneMargin = 0.995f;
// Cache-hint choices of the odd sweep in the order the autotuner tries them
// (non-temporal on every access, on none, on the aligned accesses only).
constexpr int kOddHints[3] = {1, 0, 2};

int autotune(wlb_blocks *h)
{
    h->run_shape.clear();
    if (h->slot_round != kSlotRoundMax) {  // start from the default layout
        relayout_slots(h, kSlotRoundMax);
        HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                              hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->graph_valid = false;
    }
    h->overlap = false;  // candidates first without the overlap
    float best = 1e30f;
    int bs[3] = {0, 0, 0}, bg = 0;
    // repetitions scaled so each candidate runs ~ 2e8 cell updates at most
    int reps = (int)std::max<int64_t>(2, std::min<int64_t>(10, 200000000 / std::max<int64_t>(1, 2 * h->ncells)));
    // WLB_AUTOTUNE_LOG=1 prints every candidate's time to stderr
    const char *env = getenv("WLB_AUTOTUNE_LOG");
    const bool log = env && env[0] == '1';
    // the cache hints first, on whole-row tiles with the direct odd sweep, so
    // that the shapes are compared under hints close to the final ones (the
    // hints can change a sweep's time by a third)
    {
        h->lds_stage = false;
        h->vec_want = false;
        bool pe = true;
        int po = 1;
        float bt = 1e30f;
        for (int v = 0; v < 6; ++v) {
            h->nt_even = (v & 1) == 0;
            h->nt_odd = kOddHints[v >> 1];
            int rc = set_tiles(h, 0, 0, 0, 0);
            if (rc) return rc;
            float ms = 0.f;
            rc = time_pairs(h, reps, &ms);
            if (rc) return rc;
            if (log)
                fprintf(stderr, "[wlb autotune] hints first: nt %d,%d: %.4f ms per two steps\n", h->nt_even ? 1 : 0,
                        h->nt_odd, ms);
            if (ms < kTuneMargin * bt) {
                bt = ms;
                pe = h->nt_even;
                po = h->nt_odd;
            }
        }
        h->nt_even = pe;
        h->nt_odd = po;
    }
    int blds = 0;  // odd-sweep mode: 0 direct, 1 LDS-staged, 2 row vectors
    for (int lds = 0; lds <= 2; ++lds) {
        if (lds == 2 && !(h->vec_ok && h->esize == 8)) continue;
        h->lds_stage = lds == 1;
        h->vec_want = lds == 2;
        std::vector<std::array<int, 3>> shapes;
        for (const auto &s : kShapes) shapes.push_back({s[0], s[1], s[2]});
        if (h->list_built) shapes.push_back({-1, 0, 0});
        for (const auto &s : shapes) {
            if (s[0] >= 0 && count_tiles(h, s[0], s[1], s[2]) > h->tile_cap) continue;
            for (int g : kGrids) {
                int rc = set_tiles(h, s[0], s[1], s[2], g);
                if (rc) return rc;
                if (g > 0 && g >= (int)h->tiles.size()) continue;  // same as one workgroup per tile
                if (lds == 1 && h->args.lds_stride == 0) continue;  // staging does not fit: covered by lds = 0
                if (lds == 2 && !h->args.vec_odd) continue;
                float ms = 0.f;
                rc = time_pairs(h, reps, &ms);
                if (rc) return rc;
                if (log)
                    fprintf(stderr, "[wlb autotune] tile %d,%d,%d grid %d lds %d: %zu tiles, %.4f ms per two steps\n", s[0],
                            s[1], s[2], g, lds, h->tiles.size(), ms);
                // a later candidate replaces the best only when it is faster by
                // more than the run-to-run spread of these short timings
                if (ms < kTuneMargin * best) {
                    best = ms;
                    bs[0] = s[0];
                    bs[1] = s[1];
                    bs[2] = s[2];
                    bg = g;
                    blds = lds;
                }
            }
        }
    }
    // the best shape and grid once more with each other choice of the
    // non-temporal hint per parity, for every odd-sweep kernel
    const bool ne0 = h->nt_even;  // the hints of the search above
    const int no0 = h->nt_odd;
    bool bne = ne0;
    int bno = no0;
    for (int lds = 0; lds <= 2; ++lds)
        for (int v = 0; v < 6; ++v) {
            const bool ne = (v & 1) == 0;
            const int no = kOddHints[v >> 1];
            if (ne == ne0 && no == no0) continue;  // measured above
            if (lds != 0 && no == 2) continue;  // every access of those odd sweeps is aligned: same as 1
            if (lds == 2 && !(h->vec_ok && h->esize == 8)) continue;
            h->lds_stage = lds == 1;
            h->vec_want = lds == 2;
            h->nt_even = ne;
            h->nt_odd = no;
            int rc = set_tiles(h, bs[0], bs[1], bs[2], bg);
            if (rc) return rc;
            if (lds == 1 && h->args.lds_stride == 0) continue;
            if (lds == 2 && !h->args.vec_odd) continue;
            float ms = 0.f;
            rc = time_pairs(h, reps, &ms);
            if (rc) return rc;
            if (log)
                fprintf(stderr, "[wlb autotune] tile %d,%d,%d grid %d lds %d nt %d,%d: %.4f ms per two steps\n", bs[0],
                        bs[1], bs[2], bg, lds, ne ? 1 : 0, no, ms);
            if (ms < kTuneMargin * best) {
                best = ms;
                blds = lds;
                bne = ne;
                bno = no;
            }
        }
    h->nt_even = bne;
    h->nt_odd = bno;
    h->lds_stage = blds == 1;
    h->vec_want = blds == 2;
    h->overlap = false;
    int rc = set_tiles(h, bs[0], bs[1], bs[2], bg);
    if (rc) return rc;
    // slot stride: other roundings of the large slots (the state is
    // initialised again after the autotuner, in whatever layout it keeps)
    bool big = false;
    for (int64_t s0 : h->run_slot0) big = big || s0 * h->esize >= ((int64_t)64 << 20);
    if (big) {
        size_t bround = h->slot_round;
        for (size_t cand : {(size_t)2 << 20, (size_t)0}) {
            relayout_slots(h, cand);
            HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                                  hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            h->graph_valid = false;
            float ms = 0.f;
            rc = time_pairs(h, reps, &ms);
            if (rc) return rc;
            if (log)
                fprintf(stderr, "[wlb autotune] slot stride rounding %zu KiB: %.4f ms per two steps\n", cand >> 10, ms);
            if (ms < kTuneMargin * best) {
                best = ms;
                bround = cand;
            }
        }
        relayout_slots(h, bround);
        HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                              hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->graph_valid = false;
    }
    // classes of x-runs (by y extent): every other box shape for one class
    // at a time, the other runs keeping the best shape; kept for a clear gain
    if (bs[0] >= 0 && h->rhost.size() > 1) {
        std::vector<int> ext;
        for (const HostBlock &R : h->rhost) ext.push_back(R.n[1]);
        std::sort(ext.begin(), ext.end());
        ext.erase(std::unique(ext.begin(), ext.end()), ext.end());
        if (ext.size() > 1) {
            const std::array<int, 3> glob = {bs[0], bs[1], bs[2]};
            h->run_shape.assign(h->rhost.size(), glob);
            for (int e : ext) {
                std::array<int, 3> keep = glob;
                for (const auto &c : kShapes) {
                    const std::array<int, 3> cand = {c[0], c[1], c[2]};
                    if (cand == glob) continue;
                    for (size_t r = 0; r < h->rhost.size(); ++r)
                        if (h->rhost[r].n[1] == e) h->run_shape[r] = cand;
                    if (count_tiles(h, bs[0], bs[1], bs[2]) > h->tile_cap) continue;
                    rc = set_tiles(h, bs[0], bs[1], bs[2], bg);
                    if (rc) return rc;
                    float ms = 0.f;
                    rc = time_pairs(h, reps, &ms);
                    if (rc) return rc;
                    if (log)
                        fprintf(stderr, "[wlb autotune] runs of y extent %d: tile %d,%d,%d: %.4f ms per two steps\n", e,
                                cand[0], cand[1], cand[2], ms);
                    if (ms < 0.99f * best) {
                        best = ms;
                        keep = cand;
                    }
                }
                for (size_t r = 0; r < h->rhost.size(); ++r)
                    if (h->rhost[r].n[1] == e) h->run_shape[r] = keep;
            }
            bool same = true;
            for (const auto &x : h->run_shape) same = same && x == glob;
            if (same) h->run_shape.clear();
            rc = set_tiles(h, bs[0], bs[1], bs[2], bg);
            if (rc) return rc;
        }
    }
    if (h->pull.empty() && h->push.empty()) return WLB_OK;
    // the best configuration once more with the exchange overlapped
    rc = ensure_stream2(h);
    if (rc) return rc;
    h->overlap = true;
    rc = set_tiles(h, bs[0], bs[1], bs[2], bg);
    if (rc) return rc;
    float ms = 0.f;
    rc = time_pairs(h, reps, &ms);
    if (rc) return rc;
    if (log)
        fprintf(stderr, "[wlb autotune] tile %d,%d,%d grid %d lds %d overlap 1: %.4f ms per two steps\n", bs[0], bs[1],
                bs[2], bg, blds, ms);
    if (ms < 0.99f * best) return WLB_OK;  // kept only for a clear gain (it adds launches and a second stream)
    h->overlap = false;
    return set_tiles(h, bs[0], bs[1], bs[2], bg);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *wlb_last_error(void) { return g_err.c_str(); }

int wlb_blocks_create(const wlb_block_desc *d, int32_t n, const int32_t domain[3], const int32_t periodic[3],
                      int32_t stencil, int32_t storage, size_t *arena_bytes, wlb_blocks_t *out)
{
    if (!d || n <= 0 || !domain || !periodic || !arena_bytes || !out) return fail(WLB_ERR_ARG, "null argument");
    if (stencil != WLB_D2Q9 && stencil != WLB_D3Q15 && stencil != WLB_D3Q19 && stencil != WLB_D3Q27)
        return fail(WLB_ERR_ARG, "stencil must be 9, 15, 19 or 27");
    if (storage < WLB_F64 || storage > WLB_BF16DEV) return fail(WLB_ERR_ARG, "bad storage type");
    for (int a = 0; a < 3; ++a)
        if (domain[a] <= 0 || domain[a] > 32767) return fail(WLB_ERR_ARG, "domain extent out of range");
    wlb_blocks *h = new wlb_blocks();
    h->q = stencil;
    h->storage = storage;
    h->esize = storage_esize(storage);
    for (int a = 0; a < 3; ++a) {
        h->dom[a] = domain[a];
        h->periodic[a] = periodic[a] ? 1 : 0;
    }
    // --- validate the block list: inside the domain, no overlap, full cover
    int64_t vol = 0;
    h->blocks.resize(n);
    for (int b = 0; b < n; ++b) {
        HostBlock &B = h->blocks[b];
        for (int a = 0; a < 3; ++a) {
            B.org[a] = d[b].origin[a];
            B.n[a] = d[b].size[a];
            if (B.n[a] <= 0 || B.n[a] > 32767 || B.org[a] < 0 || B.org[a] + B.n[a] > domain[a]) {
                delete h;
                return fail(WLB_ERR_ARG, "block %d outside the domain or empty", b);
            }
        }
        vol += (int64_t)B.n[0] * B.n[1] * B.n[2];
    }
    const int64_t dvol = (int64_t)domain[0] * domain[1] * domain[2];
    if (vol != dvol) {
        delete h;
        return fail(WLB_ERR_ARG, "blocks cover %lld cells, domain has %lld", (long long)vol, (long long)dvol);
    }
    for (int b = 0; b < n; ++b)
        for (int c = b + 1; c < n; ++c) {
            bool ov = true;
            for (int a = 0; a < 3; ++a) {
                const int lo = std::max(h->blocks[b].org[a], h->blocks[c].org[a]);
                const int hi = std::min(h->blocks[b].org[a] + h->blocks[b].n[a], h->blocks[c].org[a] + h->blocks[c].n[a]);
                if (lo >= hi) ov = false;
            }
            if (ov) {
                delete h;
                return fail(WLB_ERR_ARG, "blocks %d and %d overlap", b, c);
            }
        }
    h->ncells = vol;
    // --- neighbour table
    auto find_block = [&](const int p[3]) -> int {
        for (int b = 0; b < n; ++b) {
            const HostBlock &B = h->blocks[b];
            if (p[0] >= B.org[0] && p[0] < B.org[0] + B.n[0] && p[1] >= B.org[1] && p[1] < B.org[1] + B.n[1] &&
                p[2] >= B.org[2] && p[2] < B.org[2] + B.n[2])
                return b;
        }
        return -1;
    };
    for (int b = 0; b < n; ++b) {
        HostBlock &B = h->blocks[b];
        for (int k = 0; k < 27; ++k) {
            B.nbr[k] = -1;
            const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
            if (o[0] == 0 && o[1] == 0 && o[2] == 0) continue;
            int p[3];
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
                p[a] = o[a] < 0 ? B.org[a] - 1 : (o[a] > 0 ? B.org[a] + B.n[a] : B.org[a]);
                if (p[a] < 0 || p[a] >= domain[a]) {
                    if (h->periodic[a])
                        p[a] = (p[a] + domain[a]) % domain[a];
                    else
                        ok = false;
                }
            }
            if (!ok) continue;
            const int nb = find_block(p);
            if (nb < 0) {
                delete h;
                return fail(WLB_ERR_ARG, "no neighbour block for block %d offset (%d,%d,%d)", b, o[0], o[1], o[2]);
            }
            const HostBlock &N = h->blocks[nb];
            for (int a = 0; a < 3; ++a)
                if (o[a] == 0 && (N.org[a] != B.org[a] || N.n[a] != B.n[a])) {
                    delete h;
                    return fail(WLB_ERR_ARG, "blocks %d and %d do not share a whole face", b, nb);
                }
            B.nbr[k] = nb;
        }
    }
    // --- arena layout
    // Blocks that follow each other along x with the same y-z extent (an
    // x-row of a rectilinear block grid) share their population rows: row
    // (y, z) of each slot holds the cells of all blocks of the run side by
    // side, so a row of the domain is one contiguous stretch of memory.  The
    // blocks stay separate containers (own descriptor, tiles, masks, y/z
    // exchange); a population crossing an x face between two blocks of a
    // run is simply the next element of the row.  A run that spans a
    // periodic x axis wraps inside its row (no x ghost cells).
    const int align_e = 128 / h->esize;
    size_t elems = 0;
    size_t mwords = 0;
    h->dev.resize(n);
    h->nblk = n;
    std::vector<int> run_of(n, -1);
    std::vector<std::vector<int>> &runs = h->runs;
    std::vector<DevBlock> rdev;
    for (int b = 0; b < n; ++b) {
        if (run_of[b] >= 0) continue;
        // first block of the run: walk -x while the neighbour is adjacent
        // without wrapping (the face check above gives it the same y-z extent)
        int s0 = b;
        for (int guard = 0; guard < n; ++guard) {
            const int m = h->blocks[s0].nbr[12];
            if (m < 0 || m == s0 || h->blocks[m].org[0] + h->blocks[m].n[0] != h->blocks[s0].org[0]) break;
            s0 = m;
        }
        std::vector<int> r{s0};
        for (int guard = 0; guard < n; ++guard) {
            const int c = r.back(), m = h->blocks[c].nbr[14];
            if (m < 0 || m == c || h->blocks[m].org[0] != h->blocks[c].org[0] + h->blocks[c].n[0]) break;
            r.push_back(m);
        }
        for (int m : r) run_of[m] = (int)runs.size();
        runs.push_back(r);
    }
    for (const std::vector<int> &r : runs) {
        const HostBlock &F = h->blocks[r.front()], &Lb = h->blocks[r.back()];
        int W = 0, gy = 0;
        for (int m : r) {
            W += h->blocks[m].n[0];
            if (h->blocks[m].nbr[10] >= 0 || h->blocks[m].nbr[16] >= 0) gy = 1;
        }
        // the run wraps onto itself across a periodic x axis
        const bool wraps = F.nbr[12] == r.back() && Lb.nbr[14] == r.front() && F.org[0] == 0 && W == domain[0];
        // Rows of at least 256 bytes start interior x = 0 on a 128-byte
        // boundary (whole lines per wave).  Shorter rows are packed with just
        // their two ghost cells: a wave then covers several rows of nearly
        // contiguous memory instead of touching a mostly empty line per row
        // and another for each ghost cell.  A run that wraps never touches an
        // x ghost cell, so its aligned rows carry no x padding at all.  Ghost
        // rows exist only along a y face with a neighbour: beyond a wall
        // nothing is read or written (bounce-back links use the cell's own
        // slots).  Rows and planes without padding keep the sweeps' streams
        // contiguous, which measurably raises the achieved bandwidth.
        const bool packed = (size_t)W * h->esize < 256;
        const int xoff = packed ? 1 : (wraps ? 0 : align_e);
        const int pitch = packed ? W + 2
                                 : (int32_t)(wraps ? round_up((size_t)W, align_e) : round_up((size_t)align_e + W + 1, align_e));
        const int64_t plane = (int64_t)pitch * (F.n[1] + 2 * gy);
        // slot size before the stride rounding (relayout_slots places the
        // slots once every run is known)
        const int64_t slot = (int64_t)round_up((size_t)(plane * (F.n[2] + 2)), align_e);
        if (round_up((size_t)slot * h->esize, kSlotRoundMax) >= (size_t)1 << 31) {
            delete h;
            return fail(WLB_ERR_ARG, "block %d too large: one population slot must stay below 2 GiB", r.front());
        }
        h->run_slot0.push_back(slot);
        const int64_t pop = 0;
        for (size_t k = 0; k < r.size(); ++k) {
            const int b = r[k];
            const HostBlock &B = h->blocks[b];
            DevBlock &D = h->dev[b];
            std::memset(&D, 0, sizeof D);
            D.gy = gy;
            D.xoff = xoff + (B.org[0] - F.org[0]);
            D.pitch = pitch;
            D.plane = (int32_t)plane;
            D.slot = slot;
            D.pop = pop;
            for (int a = 0; a < 3; ++a) {
                D.n[a] = B.n[a];
                D.g[a] = B.org[a];
            }
            // x accesses of the run's end cells wrap by the run's length
            D.wraplo = (wraps && k == 0) ? W : 0;
            D.wraphi = (wraps && k + 1 == r.size()) ? W : 0;
            // a block that is its own neighbour on both x faces (a run of one)
            D.wrapx = (wraps && r.size() == 1) ? B.n[0] : 0;
            // blocks across an x face outside the run (none for a valid
            // rectilinear grid): read and written through their own descriptor
            D.nbx[0] = (B.nbr[12] >= 0 && run_of[B.nbr[12]] != run_of[b]) ? B.nbr[12] : -1;
            D.nbx[1] = (B.nbr[14] >= 0 && run_of[B.nbr[14]] != run_of[b]) ? B.nbr[14] : -1;
        }
        // the run as one block: the first member's rows with the run's length,
        // its x ends and the run's mask, of which every member sees its part
        DevBlock R = h->dev[r.front()];
        R.n[0] = W;
        R.xoff = xoff;
        R.wrapx = wraps ? W : 0;
        R.wraplo = R.wraphi = wraps ? W : 0;
        R.nbx[0] = h->dev[r.front()].nbx[0];
        R.nbx[1] = h->dev[r.back()].nbx[1];
        R.mpitch = (int32_t)round_up(W, 32);
        R.mplane = R.mpitch * F.n[1];
        R.mask = (int64_t)mwords;  // provisional; -1 if the run has no solid nearby (set at init)
        mwords += (size_t)R.mplane * F.n[2];
        for (int m : r) {
            DevBlock &D = h->dev[m];
            D.mpitch = R.mpitch;
            D.mplane = R.mplane;
            D.mask = R.mask + (h->blocks[m].org[0] - F.org[0]);
        }
        rdev.push_back(R);
        HostBlock RH = F;
        RH.n[0] = W;
        for (int k = 0; k < 27; ++k) RH.nbr[k] = -1;
        RH.nbr[12] = F.nbr[12];
        RH.nbr[14] = Lb.nbr[14];
        for (int m : r)
            for (int k : {4, 10, 16, 22})
                if (h->blocks[m].nbr[k] >= 0) RH.nbr[k] = h->blocks[m].nbr[k];
        h->rhost.push_back(RH);
    }
    h->dev.insert(h->dev.end(), rdev.begin(), rdev.end());
    elems = relayout_slots(h, kSlotRoundMax);
    size_t off = 0;
    h->off_pop = off;
    h->pop_bytes = round_up(elems * h->esize, 256);
    off += h->pop_bytes;
    h->off_mask = off;
    h->mask_words = mwords;
    off += round_up(mwords * 4, 256);
    h->off_blocks = off;
    off += round_up(h->dev.size() * sizeof(DevBlock), 256);
    size_t cap = 0;
    for (const auto &s : kShapes)
        cap = std::max(cap, std::max(count_tiles(h, s[0], s[1], s[2]), count_tiles(h, s[0], s[1], s[2], true)));
    h->tile_cap = cap;
    h->off_tiles = off;
    off += round_up(cap * sizeof(int4), 256);
    // fluid-cell lists (every interior cell at most once) and their tiles
    h->list_ok = true;
    for (const HostBlock &B : h->rhost)
        if (B.n[0] > 1024 || B.n[1] > 1024 || B.n[2] > 4096) h->list_ok = false;
    if (h->list_ok) {
        h->off_cells = off;
        off += round_up((size_t)h->ncells * 4, 256);
        h->ltile_cap = (size_t)h->ncells / kWG + 2 * h->rhost.size() + 1;  // interior and frontier lists per run
        h->off_ltiles = off;
        off += round_up(h->ltile_cap * sizeof(int4), 256);
    }
    // row tiles of the vector odd sweep (at most one per row)
    h->vtile_cap = 1;
    for (const HostBlock &B : h->rhost) h->vtile_cap += (size_t)B.n[1] * B.n[2];
    h->off_vtiles = off;
    off += round_up(h->vtile_cap * sizeof(int4), 256);
    // --- exchange work lists
    // Items of one y/z face (or edge) direction k of descriptor a (extent
    // and neighbour flags A) with neighbour descriptor nbd (extent Bn).
    auto add_items = [&](const HostBlock &A, int a_id, const HostBlock &Bn, int nb_id, int k) {
        // x neighbours (the block itself or another) are addressed directly
        // by the kernels: no x items, and y/z regions reach the x ends of
        // the rows on every side that has a neighbour
        const bool xlo = A.nbr[12] >= 0, xhi = A.nbr[14] >= 0;
        const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
        for (int j = 1; j < stencil; ++j) {
            bool in = true;
            for (int a = 0; a < 3; ++a)
                if (o[a] != 0 && ccq(stencil, j, a) != o[a]) in = false;
            if (!in) continue;
            // Cells of the ghost region on side o for which population j is
            // used: the cell g - c_j that reads it (after the even sweep) or
            // writes it (after the odd sweep) must be an interior cell of A.
            // Along the shared axes (o_a = 0) this shrinks the region by one
            // cell on the side c_j points from; it also makes every interior
            // (cell, slot) of the neighbour the target of exactly one copy
            // after the odd sweep.
            int ext[3], ghost0[3], inner0[3];
            for (int a = 0; a < 3; ++a) {
                if (o[a] != 0) {
                    ext[a] = 1;
                    ghost0[a] = o[a] < 0 ? -1 : A.n[a];
                    inner0[a] = o[a] < 0 ? Bn.n[a] - 1 : 0;
                } else if (a == 0) {
                    // the reader / writer g - c_j may sit across an x face
                    // with a neighbour; only a face without one limits the range
                    const int lo = (ccq(stencil, j, 0) > 0 && !xlo) ? 1 : 0;
                    const int hi = (ccq(stencil, j, 0) < 0 && !xhi) ? A.n[0] - 1 : A.n[0];
                    ext[a] = hi - lo;
                    ghost0[a] = lo;
                    inner0[a] = lo;
                } else {
                    const int lo = std::max(0, ccq(stencil, j, a)), hi = std::min(A.n[a], A.n[a] + ccq(stencil, j, a));
                    ext[a] = hi - lo;
                    ghost0[a] = lo;
                    inner0[a] = lo;
                }
            }
            const int cells = ext[0] * ext[1] * ext[2];
            for (int s0 = 0; s0 < cells; s0 += kXChunk) {
                XItem it;
                it.slot = j;
                it.ex = ext[0];
                it.ey = ext[1];
                it.start = s0;
                it.count = std::min(kXChunk, cells - s0);
                // after the even sweep: neighbour interior -> own ghost layer
                it.sb = nb_id;
                it.db = a_id;
                it.chk = -1;
                for (int a = 0; a < 3; ++a) {
                    it.s0[a] = inner0[a];
                    it.d0[a] = ghost0[a];
                }
                h->pull.push_back(it);
                // after the odd sweep: own ghost layer -> neighbour interior,
                // unless the writer (neighbour cell - c_j) is solid
                it.sb = a_id;
                it.db = nb_id;
                it.chk = opp(j);
                for (int a = 0; a < 3; ++a) {
                    it.s0[a] = ghost0[a];
                    it.d0[a] = inner0[a];
                }
                h->push.push_back(it);
                h->xchg_elems += it.count;
            }
        }
    };
    // Per x-run and direction: where the neighbour of every block of the run
    // is the block at the same place in one other run (a rectilinear grid),
    // the run exchanges whole domain rows through the run descriptors;
    // otherwise each block exchanges its own piece.
    for (size_t r = 0; r < runs.size(); ++r) {
        const std::vector<int> &mem = runs[r];
        for (int k = 0; k < 27; ++k) {
            if (k % 3 != 1) continue;  // o_x = 0: y/z faces and y-z edges only
            const int nb0 = h->blocks[mem.front()].nbr[k];
            bool whole = nb0 >= 0 && runs[run_of[nb0]].size() == mem.size();
            for (size_t i = 0; i < mem.size() && whole; ++i)
                whole = h->blocks[mem[i]].nbr[k] == runs[run_of[nb0]][i];
            if (whole) {
                const int r2 = run_of[nb0];
                add_items(h->rhost[r], n + (int)r, h->rhost[r2], n + r2, k);
            } else {
                for (int m : mem)
                    if (h->blocks[m].nbr[k] >= 0) add_items(h->blocks[m], m, h->blocks[h->blocks[m].nbr[k]], h->blocks[m].nbr[k], k);
            }
        }
    }
    h->off_pull = off;
    off += round_up(h->pull.size() * sizeof(XItem) + 1, 256);
    h->off_push = off;
    off += round_up(h->push.size() * sizeof(XItem) + 1, 256);
    h->off_partials = off;
    off += round_up(cap * 8 * sizeof(double), 256);
    h->off_totals = off;
    off += 256;
    h->off_mlp = off;
    off += round_up(mlp_dev_bytes(), 256);
    const size_t plane_cells = (size_t)domain[0] * domain[1];
    size_t stage = (size_t)64 << 20;
    stage = std::max(stage, (size_t)dvol);                            // solid array
    stage = std::max(stage, plane_cells * 4 * sizeof(double));        // rho, u of one plane
    stage = std::max(stage, plane_cells * stencil * sizeof(double));  // populations of one plane
    h->stage_bytes = round_up(stage, 256);
    h->off_stage = off;
    off += h->stage_bytes;
    h->arena_bytes = off;
    build_tiles(h, 0, 0, 0, h->tiles);
    *arena_bytes = off;
    *out = h;
    return WLB_OK;
}

int wlb_blocks_bind(wlb_blocks_t h, void *arena, size_t bytes, void *stream)
{
    if (!h || !arena) return fail(WLB_ERR_ARG, "null argument");
    if (!stream) return fail(WLB_ERR_ARG, "a non-null HIP stream is required");
    if (bytes < h->arena_bytes) return fail(WLB_ERR_ARG, "arena of %zu bytes < required %zu", bytes, h->arena_bytes);
    if (((uintptr_t)arena) % 256) return fail(WLB_ERR_ARG, "arena must be 256-byte aligned");
    h->arena = static_cast<char *>(arena);
    h->stream = static_cast<hipStream_t>(stream);
    drop_graph(h);
    HIPCHK(hipMemsetAsync(h->arena, 0, h->off_blocks, h->stream));  // populations and masks
    HIPCHK(hipMemcpyAsync(h->arena + h->off_pull, h->pull.data(), h->pull.size() * sizeof(XItem),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->arena + h->off_push, h->push.data(), h->push.size() * sizeof(XItem),
                          hipMemcpyHostToDevice, h->stream));
    h->bound = true;
    if (h->overlap) {
        int rc = ensure_stream2(h);
        if (rc) return rc;
    }
    h->args.arena = h->arena + h->off_pop;
    h->args.blocks = reinterpret_cast<const DevBlock *>(h->arena + h->off_blocks);
    h->args.tiles = reinterpret_cast<const int4 *>(h->arena + h->off_tiles);
    h->args.cells = reinterpret_cast<const uint32_t *>(h->arena + h->off_cells);
    h->args.masks = reinterpret_cast<const uint32_t *>(h->arena + h->off_mask);
    h->args.mlp = h->arena + h->off_mlp;
    for (int a = 0; a < 3; ++a) h->args.dom[a] = h->dom[a];
    h->args.periodic = h->periodic[0] | (h->periodic[1] << 1) | (h->periodic[2] << 2);
    HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                          hipMemcpyHostToDevice, h->stream));
    return upload_tiles(h);
}

int wlb_lbm_init(wlb_blocks_t h, int32_t collision, const wlb_lbm_params *p, const double *rho, const double *u,
                 const uint8_t *solid)
{
    if (!h || !p || !rho || !u) return fail(WLB_ERR_ARG, "null argument");
    if (!h->bound) return fail(WLB_ERR_STATE, "wlb_blocks_bind must come first");
    if (collision < WLB_SRT || collision > WLB_CUMULANT) return fail(WLB_ERR_ARG, "bad collision operator");
    if (collision >= WLB_KBC && h->q != WLB_D3Q27)
        return fail(WLB_ERR_UNSUPPORTED, "KBC and the cumulant collision run with D3Q27");
    if (collision == WLB_MRT && h->q != WLB_D3Q19 && h->q != WLB_D3Q27)
        return fail(WLB_ERR_UNSUPPORTED, "MRT runs with D3Q19 and D3Q27");
    if (!(p->tau > 0.5)) return fail(WLB_ERR_ARG, "tau must exceed 1/2");
    if (collision == WLB_TRT && !(p->magic > 0.0)) return fail(WLB_ERR_ARG, "TRT needs magic > 0");
    if (p->pressure_axis < -1 || p->pressure_axis > 2) return fail(WLB_ERR_ARG, "bad pressure axis");
    if (p->pressure_axis >= 0 && h->periodic[p->pressure_axis])
        return fail(WLB_ERR_ARG, "the pressure axis must not be periodic");
    if (p->closure < WLB_CLOSURE_NONE || p->closure > WLB_CLOSURE_MLP) return fail(WLB_ERR_ARG, "bad closure");
    if (p->closure == WLB_CLOSURE_MLP) {
        if (!p->mlp) return fail(WLB_ERR_ARG, "the MLP closure needs weights");
        if (h->q != WLB_D3Q19 || collision >= WLB_MRT || h->storage == WLB_F64)
            return fail(WLB_ERR_UNSUPPORTED, "the MLP closure runs with D3Q19 SRT/TRT and FP32/FP16/BF16 storage");
    }
    h->collision = collision;
    h->params = *p;
    drop_graph(h);
    SweepArgs &a = h->args;
    a.pressure_axis = p->pressure_axis;
    a.closure = p->closure;
    a.omega = 1.0 / p->tau;
    a.magic = p->magic;
    a.omega_minus = collision == WLB_TRT ? 1.0 / (0.5 + p->magic / (p->tau - 0.5)) : a.omega;
    a.omega_bulk = p->omega_bulk;
    a.omega_higher = p->omega_higher;
    for (int k = 0; k < 3; ++k) a.force[k] = p->force[k];
    a.rho_in = p->rho_in;
    a.rho_out = p->rho_out;
    a.tau0 = p->tau;
    a.smag_k = 18.0 * std::sqrt(2.0) * p->cs_smag * p->cs_smag;
    if (p->closure == WLB_CLOSURE_MLP) {
        std::vector<unsigned char> dev(mlp_dev_bytes());
        mlp_prepare(p->mlp, dev.data());
        HIPCHK(hipMemcpyAsync(h->arena + h->off_mlp, dev.data(), dev.size(), hipMemcpyHostToDevice, h->stream));
    }
    // --- geometry: which blocks need masks, then build them on the device
    const int64_t plane = (int64_t)h->dom[0] * h->dom[1];
    const int64_t N = plane * h->dom[2];
    int64_t nsolid = 0;
    if (solid)
        for (int64_t k = 0; k < N; ++k) nsolid += solid[k] ? 1 : 0;
    h->nfluid = N - nsolid;
    int64_t mwords = 0;
    for (size_t r = 0; r < h->rhost.size(); ++r) {
        const HostBlock &B = h->rhost[r];
        DevBlock &D = h->dev[h->nblk + r];
        bool need = false;
        if (solid && nsolid > 0) {
            for (int z = -1; z <= B.n[2] && !need; ++z)
                for (int y = -1; y <= B.n[1] && !need; ++y)
                    for (int x = -1; x <= B.n[0] && !need; ++x) {
                        int g[3] = {B.org[0] + x, B.org[1] + y, B.org[2] + z};
                        bool ok = true;
                        for (int ax = 0; ax < 3; ++ax)
                            if (g[ax] < 0 || g[ax] >= h->dom[ax]) {
                                if (h->periodic[ax])
                                    g[ax] = (g[ax] + h->dom[ax]) % h->dom[ax];
                                else
                                    ok = false;
                            }
                        if (ok && solid[(g[2] * (int64_t)h->dom[1] + g[1]) * h->dom[0] + g[0]]) need = true;
                    }
        }
        D.mask = need ? mwords : -1;
        mwords += (int64_t)D.mplane * B.n[2];
        for (int m : h->runs[r])
            h->dev[m].mask = need ? D.mask + (h->blocks[m].org[0] - B.org[0]) : -1;
    }
    HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemsetAsync(h->arena + h->off_pop, 0, h->pop_bytes, h->stream));
    if (solid && nsolid > 0) {
        if ((size_t)N > h->stage_bytes) return fail(WLB_ERR_ARG, "staging too small for the solid array");
        HIPCHK(hipMemcpyAsync(h->arena + h->off_stage, solid, N, hipMemcpyHostToDevice, h->stream));
        HIPCHK(launch_masks(h->args, reinterpret_cast<const uint8_t *>(h->arena + h->off_stage), h->q, aux_grid(h),
                            h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    // fluid-cell lists for list tiles
    h->list_built = false;
    h->ltiles.clear();
    if (solid && nsolid > 0 && h->list_ok) {
        // interior cells of every block first, then the frontier cells (the
        // split that the interior/frontier overlap launches separately)
        std::vector<uint32_t> cells;
        cells.reserve((size_t)h->nfluid);
        for (int pass = 0; pass < 2; ++pass) {
            for (size_t r = 0; r < h->rhost.size(); ++r) {
                const HostBlock &B = h->rhost[r];
                const int b = h->nblk + (int)r;
                int y0, y1, z0, z1;
                interior_rows(B, y0, y1, z0, z1);
                const size_t first = cells.size();
                for (int z = 0; z < B.n[2]; ++z)
                    for (int y = 0; y < B.n[1]; ++y) {
                        if (in_interior(y, z, y0, y1, z0, z1) != (pass == 0)) continue;
                        for (int x = 0; x < B.n[0]; ++x) {
                            const int64_t g = ((int64_t)(B.org[2] + z) * h->dom[1] + (B.org[1] + y)) * h->dom[0] +
                                              (B.org[0] + x);
                            if (!solid[g]) cells.push_back((uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20));
                        }
                    }
                for (size_t k = first; k < cells.size(); k += kWG)
                    h->ltiles.push_back(
                        make_int4((int)b, (int)k, 0, -(int)std::min<size_t>(kWG, cells.size() - k)));
            }
            if (pass == 0) h->nint_ltiles = (int)h->ltiles.size();
        }
        if (h->ltiles.size() <= h->ltile_cap && !cells.empty()) {
            HIPCHK(hipMemcpyAsync(h->arena + h->off_cells, cells.data(), cells.size() * 4, hipMemcpyHostToDevice,
                                  h->stream));
            HIPCHK(hipMemcpyAsync(h->arena + h->off_ltiles, h->ltiles.data(), h->ltiles.size() * sizeof(int4),
                                  hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            h->list_built = true;
        } else {
            h->ltiles.clear();
        }
    }
    {
        const int rcv = build_vtiles(h);
        if (rcv) return rcv;
    }
    if (h->list_mode && !h->list_built) {
        const int rc0 = set_tiles(h, 0, 0, 0, h->grid);
        if (rc0) return rc0;
    } else {
        const int rc0 = upload_tiles(h);  // list tiles may have changed
        if (rc0) return rc0;
    }
    int rc = do_init_state(h, rho, u);
    if (rc) return rc;
    h->inited = true;
    if (p->autotune) {
        rc = autotune(h);
        if (rc) return rc;
        rc = do_init_state(h, rho, u);
        if (rc) return rc;
    }
    return WLB_OK;
}

int wlb_lbm_sweep(wlb_blocks_t h)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->pending) return fail(WLB_ERR_STATE, "wlb_ghost_exchange is due before the next sweep");
    const bool odd = h->parity == 1;
    int rc = run_sweep(h, odd);
    if (rc) return rc;
    h->pending = odd ? 2 : 1;
    h->parity ^= 1;
    h->last_sweep = odd ? 1 : 0;
    h->steps += 1;
    return WLB_OK;
}

int wlb_ghost_exchange(wlb_blocks_t h)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    // the exchange after the last sweep: pull after an even sweep (layout now
    // swapped), push after an odd one (layout natural)
    if (!h->pending && h->last_sweep < 0) return WLB_OK;  // nothing swept since init / set
    const bool after_odd = h->pending ? (h->pending == 2) : (h->last_sweep == 1);
    int rc = run_exchange(h, after_odd);
    if (rc) return rc;
    h->pending = 0;
    return WLB_OK;
}

int wlb_lbm_step(wlb_blocks_t h, int32_t nsteps)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (nsteps < 0) return fail(WLB_ERR_ARG, "negative step count");
    int rc;
    if (h->pending) {
        rc = wlb_ghost_exchange(h);
        if (rc) return rc;
    }
    const int he = h->params.health_every;
    while (nsteps > 0) {
        const int64_t before = h->steps;
        if (h->parity == 1 || nsteps < 2 || !h->use_graph || h->timing) {
            rc = one_step(h);
            if (rc) return rc;
            nsteps -= 1;
        } else {
            if (!h->graph_valid) {
                rc = capture_graph(h);
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(h->gexec, h->stream));
            h->last_sweep = 1;
            h->steps += 2;
            nsteps -= 2;
        }
        if (he > 0 && (h->steps / he) != (before / he)) {
            rc = health_check(h);
            if (rc) return rc;
        }
    }
    return WLB_OK;
}

int wlb_moments_get(wlb_blocks_t h, double *rho, double *u, double totals[8])
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->pending) {
        int rc = wlb_ghost_exchange(h);
        if (rc) return rc;
    }
    if (totals) {
        int rc = compute_totals(h, totals);
        if (rc) return rc;
    }
    if (rho || u) {
        const int64_t plane = (int64_t)h->dom[0] * h->dom[1];
        const int64_t N = plane * h->dom[2];
        const int kz = planes_per_chunk(h, 4 * sizeof(double));
        double *stage = reinterpret_cast<double *>(h->arena + h->off_stage);
        for (int z0 = 0; z0 < h->dom[2]; z0 += kz) {
            const int z1 = std::min(h->dom[2], z0 + kz);
            const int64_t S = (int64_t)(z1 - z0) * plane;
            MomArgs m{};
            m.s = h->args;
            m.swapped = h->parity;
            m.z0 = z0;
            m.z1 = z1;
            m.out = stage;
            m.partials = nullptr;
            HIPCHK(moments_dispatch(h, m, aux_grid(h)));
            if (rho) HIPCHK(hipMemcpyAsync(rho + z0 * plane, stage, S * sizeof(double), hipMemcpyDeviceToHost, h->stream));
            if (u)
                for (int a = 0; a < 3; ++a)
                    HIPCHK(hipMemcpyAsync(u + a * N + z0 * plane, stage + (1 + a) * S, S * sizeof(double),
                                          hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        }
    }
    return WLB_OK;
}

int wlb_force_get(wlb_blocks_t h, double out[8])
{
    if (!h || !out) return fail(WLB_ERR_ARG, "null argument");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->steps == 0) return fail(WLB_ERR_STATE, "no step since wlb_lbm_init: the force is that of the last step");
    double *partials = reinterpret_cast<double *>(h->arena + h->off_partials);
    HIPCHK(force_dispatch(h, partials, aux_grid(h)));
    double *tot = reinterpret_cast<double *>(h->arena + h->off_totals);
    HIPCHK(launch_reduce_sum8(partials, (int)h->tiles.size(), tot, h->stream));
    HIPCHK(hipMemcpyAsync(out, tot, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return WLB_OK;
}

int wlb_debug_write_coverage(wlb_blocks_t h, int32_t odd, uint32_t *counts)
{
    if (!h || !counts) return fail(WLB_ERR_ARG, "null argument");
    if (odd != 0 && odd != 1) return fail(WLB_ERR_ARG, "odd must be 0 or 1");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->storage != WLB_F32) return fail(WLB_ERR_UNSUPPORTED, "the write-coverage check runs on FP32 storage");
    HIPCHK(hipMemsetAsync(h->arena + h->off_pop, 0, h->pop_bytes, h->stream));
    h->inited = false;  // the populations now hold counters
    h->cover = true;
    const int rc = enqueue_step(h, odd != 0);
    h->cover = false;
    if (rc) return rc;
    std::vector<uint32_t> raw(h->pop_bytes / sizeof(uint32_t));
    HIPCHK(hipMemcpyAsync(raw.data(), h->arena + h->off_pop, h->pop_bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const int64_t nx = h->dom[0], ny = h->dom[1], N = nx * ny * h->dom[2];
    std::fill(counts, counts + (int64_t)h->q * N, 0u);
    for (int b = 0; b < h->nblk; ++b) {
        const DevBlock &B = h->dev[b];
        for (int i = 0; i < h->q; ++i)
            for (int z = 0; z < B.n[2]; ++z)
                for (int y = 0; y < B.n[1]; ++y)
                    for (int x = 0; x < B.n[0]; ++x)
                        counts[i * N + ((int64_t)(B.g[2] + z) * ny + B.g[1] + y) * nx + B.g[0] + x] =
                            raw[B.pop + i * B.slot + (int64_t)(z + 1) * B.plane + (int64_t)(y + B.gy) * B.pitch + B.xoff + x];
    }
    return WLB_OK;
}

static int pdfs_io(wlb_blocks_t h, double *d, bool to_dev)
{
    if (!h || !d) return fail(WLB_ERR_ARG, "null argument");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->pending) {
        int rc = wlb_ghost_exchange(h);
        if (rc) return rc;
    }
    const int64_t plane = (int64_t)h->dom[0] * h->dom[1];
    const int64_t N = plane * h->dom[2];
    const int kz = planes_per_chunk(h, h->q * sizeof(double));
    double *stage = reinterpret_cast<double *>(h->arena + h->off_stage);
    for (int z0 = 0; z0 < h->dom[2]; z0 += kz) {
        const int z1 = std::min(h->dom[2], z0 + kz);
        const int64_t S = (int64_t)(z1 - z0) * plane;
        if (to_dev) {
            for (int i = 0; i < h->q; ++i)
                HIPCHK(hipMemcpyAsync(stage + i * S, d + i * N + z0 * plane, S * sizeof(double),
                                      hipMemcpyHostToDevice, h->stream));
            HIPCHK(pdfs_dispatch(h, stage, z0, z1, true, false, aux_grid(h)));
        } else {
            HIPCHK(pdfs_dispatch(h, stage, z0, z1, false, h->parity == 1, aux_grid(h)));
            for (int i = 0; i < h->q; ++i)
                HIPCHK(hipMemcpyAsync(d + i * N + z0 * plane, stage + i * S, S * sizeof(double),
                                      hipMemcpyDeviceToHost, h->stream));
        }
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (to_dev) {
        h->parity = 0;
        h->pending = 0;
        h->last_sweep = -1;
    }
    return WLB_OK;
}

int wlb_pdfs_get(wlb_blocks_t h, double *d) { return pdfs_io(h, d, false); }
int wlb_pdfs_set(wlb_blocks_t h, const double *d) { return pdfs_io(h, const_cast<double *>(d), true); }

int wlb_info(wlb_blocks_t h, wlb_info_t *o)
{
    if (!h || !o) return fail(WLB_ERR_ARG, "null argument");
    o->steps = h->steps;
    o->parity = h->parity;
    o->n_blocks = (int32_t)h->blocks.size();
    o->n_cells = h->ncells;
    o->n_fluid = h->inited ? h->nfluid : h->ncells;
    o->n_tiles = (int32_t)(h->list_mode ? h->ltiles.size() : h->tiles.size());
    for (int a = 0; a < 3; ++a) o->tile[a] = h->shape[a];
    {
        std::vector<int> cls;
        for (size_t r = 0; r < h->run_shape.size(); ++r)
            if (h->run_shape[r] != std::array<int, 3>{h->shape[0], h->shape[1], h->shape[2]}) cls.push_back(h->rhost[r].n[1]);
        std::sort(cls.begin(), cls.end());
        o->n_class_tiles = (int32_t)(std::unique(cls.begin(), cls.end()) - cls.begin());
    }
    o->slot_round_kib = (int32_t)(h->slot_round >> 10);
    o->grid = h->grid;
    o->lds_staging = (h->args.vec_odd && h->esize == 8) ? 2 : (h->args.lds_stride > 0 ? 1 : 0);
    o->overlap = split_sweeps(h) ? 1 : 0;
    o->nt_even = h->nt_even ? 1 : 0;
    o->nt_odd = h->nt_odd;
    o->n_xchg_items = (int32_t)h->pull.size();
    o->xchg_elems = h->xchg_elems;
    o->arena_bytes = h->arena_bytes;
    o->pop_bytes = h->pop_bytes;
    return WLB_OK;
}

int wlb_set_tiles(wlb_blocks_t h, int32_t tx, int32_t ty, int32_t tz, int32_t grid)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (tx < -1 || ty < 0 || tz < 0) return fail(WLB_ERR_ARG, "negative tile shape");
    if (grid < -1) return fail(WLB_ERR_ARG, "grid must be -1, 0 or a workgroup count");
    if (tx > 0 && (ty < 1 || tz < 1 || (int64_t)tx * ty * tz > kWG))
        return fail(WLB_ERR_ARG, "tile shape must have at most %d cells", kWG);
    h->run_shape.clear();
    return set_tiles(h, tx, ty, tz, grid);
}

int wlb_set_class_tiles(wlb_blocks_t h, int32_t y_extent, int32_t tx, int32_t ty, int32_t tz)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (tx < 0 || ty < 0 || tz < 0) return fail(WLB_ERR_ARG, "negative tile shape");
    if (tx > 0 && (int64_t)tx * std::max(ty, 1) * std::max(tz, 1) > kWG)
        return fail(WLB_ERR_ARG, "tile shape must have at most %d cells", kWG);
    if (h->list_mode || h->shape[0] < 0) return fail(WLB_ERR_STATE, "fluid-cell list tiles are in use");
    bool any = false;
    for (const HostBlock &R : h->rhost) any = any || R.n[1] == y_extent;
    if (!any) return fail(WLB_ERR_ARG, "no x-run has y extent %d", y_extent);
    std::vector<std::array<int, 3>> prev = h->run_shape;
    if (h->run_shape.empty()) h->run_shape.assign(h->rhost.size(), {h->shape[0], h->shape[1], h->shape[2]});
    for (size_t r = 0; r < h->rhost.size(); ++r)
        if (h->rhost[r].n[1] == y_extent) h->run_shape[r] = {tx, ty, tz};
    if (count_tiles(h, h->shape[0], h->shape[1], h->shape[2], h->overlap) > h->tile_cap) {
        h->run_shape.swap(prev);
        return fail(WLB_ERR_ARG, "these tile shapes yield more tiles than the tile table holds");
    }
    return set_tiles(h, h->shape[0], h->shape[1], h->shape[2], h->grid);
}

int wlb_set_slot_round(wlb_blocks_t h, int32_t kib)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (kib != 16384 && kib != 2048 && kib != 0) return fail(WLB_ERR_ARG, "slot rounding must be 16384, 2048 or 0 KiB");
    if (h->inited) return fail(WLB_ERR_STATE, "the slot stride is set before wlb_lbm_init");
    relayout_slots(h, (size_t)kib << 10);
    if (h->bound) {
        HIPCHK(hipMemcpyAsync(h->arena + h->off_blocks, h->dev.data(), h->dev.size() * sizeof(DevBlock),
                              hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->graph_valid = false;
    return WLB_OK;
}

int wlb_set_nontemporal(wlb_blocks_t h, int32_t even, int32_t odd)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (odd < 0 || odd > 2) return fail(WLB_ERR_ARG, "odd-sweep hint must be 0, 1 or 2");
    h->nt_even = even != 0;
    h->nt_odd = odd;
    h->graph_valid = false;  // the captured launches hold the old arguments
    return WLB_OK;
}

int wlb_set_lds_staging(wlb_blocks_t h, int32_t on)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (on < 0 || on > 2) return fail(WLB_ERR_ARG, "odd-sweep mode must be 0, 1 or 2");
    h->lds_stage = on == 1;
    h->vec_want = on == 2;
    update_lds_stride(h);
    return WLB_OK;
}

int wlb_set_overlap(wlb_blocks_t h, int32_t on)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (on && h->bound) {
        int rc = ensure_stream2(h);
        if (rc) return rc;
    }
    h->overlap = on != 0;
    h->graph_valid = false;
    return set_tiles(h, h->shape[0], h->shape[1], h->shape[2], h->grid);
}

int wlb_set_graph(wlb_blocks_t h, int32_t on)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    h->use_graph = on != 0;
    return WLB_OK;
}

int wlb_set_kernel_timing(wlb_blocks_t h, int32_t on)
{
    if (!h) return fail(WLB_ERR_ARG, "null handle");
    if (h->timing) {
        int rc = fold_events(h);
        if (rc) return rc;
    }
    h->timing = on != 0;
    for (int k = 0; k < 4; ++k) {
        h->ms[k] = 0.0;
        h->cnt[k] = 0;
    }
    return WLB_OK;
}

int wlb_kernel_times(wlb_blocks_t h, double ms[4], int64_t launches[4])
{
    if (!h || !ms || !launches) return fail(WLB_ERR_ARG, "null argument");
    int rc = fold_events(h);
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) {
        ms[k] = h->ms[k];
        launches[k] = h->cnt[k];
    }
    return WLB_OK;
}

void wlb_blocks_destroy(wlb_blocks_t h)
{
    if (!h) return;
    if (h->stream) hipStreamSynchronize(h->stream);
    if (h->stream2) hipStreamSynchronize(h->stream2);
    drop_graph(h);
    if (h->stream2) hipStreamDestroy(h->stream2);
    if (h->ev_fork) hipEventDestroy(h->ev_fork);
    if (h->ev_join) hipEventDestroy(h->ev_join);
    for (auto &e : h->ev_pool) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    delete h;
}

int wlb_box_filter(wlb_blocks_t h, int32_t factor, double *out)
{
    if (!h || !out) return fail(WLB_ERR_ARG, "null argument");
    if (!h->inited) return fail(WLB_ERR_STATE, "wlb_lbm_init must come first");
    if (h->blocks.size() != 1) return fail(WLB_ERR_UNSUPPORTED, "the box filter works on single-block handles");
    if (factor < 1) return fail(WLB_ERR_ARG, "filter factor must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (h->dom[a] % factor) return fail(WLB_ERR_ARG, "the filter factor must divide the domain");
    if (h->pending) {
        int rc = wlb_ghost_exchange(h);
        if (rc) return rc;
    }
    const int64_t nc = (int64_t)(h->dom[0] / factor) * (h->dom[1] / factor) * (h->dom[2] / factor);
    const bool sw = h->parity == 1;
    hipError_t e;
    switch (h->storage) {
    case WLB_F64: e = filter_f64(h->q, h->args, factor, out, nc, sw, h->stream); break;
    case WLB_F32: e = filter_f32(h->q, h->args, factor, out, nc, sw, h->stream); break;
    case WLB_F16DEV: e = filter_f16(h->q, h->args, factor, out, nc, sw, h->stream); break;
    default: e = filter_bf16(h->q, h->args, factor, out, nc, sw, h->stream); break;
    }
    HIPCHK(e);
    HIPCHK(hipStreamSynchronize(h->stream));
    return WLB_OK;
}

int wlb_les_targets(const double *filt, const int32_t nc[3], double tau0, float *raw, float *target, void *stream)
{
    if (!filt || !nc || !raw || !target) return fail(WLB_ERR_ARG, "null argument");
    for (int a = 0; a < 3; ++a)
        if (nc[a] < 3) return fail(WLB_ERR_ARG, "coarse grid must have at least 3 cells per axis");
    HIPCHK(launch_les_targets(filt, nc, tau0, raw, target, static_cast<hipStream_t>(stream)));
    return WLB_OK;
}

int wlb_mlp_forward(const float *params, void *workspace, const float *raw, int64_t n, float *out, int32_t *fallback,
                    void *stream)
{
    if (!params || !workspace || (n > 0 && (!raw || !out || !fallback))) return fail(WLB_ERR_ARG, "null argument");
    if (n < 0) return fail(WLB_ERR_ARG, "negative sample count");
    if (((uintptr_t)workspace) % 16) return fail(WLB_ERR_ARG, "workspace must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<unsigned char> dev(mlp_dev_bytes());
    mlp_prepare(params, dev.data());
    HIPCHK(hipMemcpyAsync(workspace, dev.data(), dev.size(), hipMemcpyHostToDevice, st));
    if (n > 0) HIPCHK(launch_mlp_forward(workspace, raw, n, out, fallback, st));
    HIPCHK(hipStreamSynchronize(st));
    return WLB_OK;
}

size_t wlb_mlp_grad_workspace(int64_t n) { return n > 0 ? mlp_grad_workspace_bytes(n) : 0; }

int wlb_mlp_grad(const float *params, const float *raw, const float *target, int64_t n, double inv_scale, float *grad,
                 float *loss, void *workspace, size_t ws_bytes, void *stream)
{
    if (!params || !raw || !target || !grad || !loss || !workspace) return fail(WLB_ERR_ARG, "null argument");
    if (n <= 0) return fail(WLB_ERR_ARG, "empty minibatch");
    if (ws_bytes < mlp_grad_workspace_bytes(n)) return fail(WLB_ERR_ARG, "workspace too small");
    HIPCHK(launch_mlp_grad(params, raw, target, n, (float)inv_scale, grad, loss, static_cast<float *>(workspace),
                           static_cast<hipStream_t>(stream)));
    return WLB_OK;
}

int wlb_mlp_grad_noalloc(const float *params, const float *raw, const float *target, int64_t n, double inv_scale,
                         float *grad, float *loss, void *stream)
{
    if (!params || !raw || !target || !grad || !loss) return fail(WLB_ERR_ARG, "null argument");
    if (n <= 0) return fail(WLB_ERR_ARG, "empty minibatch");
    if (n > WLB_MLP_NOALLOC_MAX_SAMPLES)
        return fail(WLB_ERR_ARG, "minibatch of %lld samples exceeds the %d that the library's fixed scratch holds",
                    (long long)n, WLB_MLP_NOALLOC_MAX_SAMPLES);
    void *scr = nullptr;
    HIPCHK(mlp_scratch_address(&scr));
    HIPCHK(launch_mlp_grad(params, raw, target, n, (float)inv_scale, grad, loss, static_cast<float *>(scr),
                           static_cast<hipStream_t>(stream)));
    return WLB_OK;
}

int wlb_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr, double beta1,
                 double beta2, double eps, void *stream)
{
    if (!params || !grad || !m || !v) return fail(WLB_ERR_ARG, "null argument");
    if (step < 1) return fail(WLB_ERR_ARG, "Adam step count starts at 1");
    HIPCHK(launch_mlp_adam(params, grad, m, v, step, (float)lr, (float)beta1, (float)beta2, (float)eps,
                           static_cast<hipStream_t>(stream)));
    return WLB_OK;
}

int wlb_copy_probe(void *dst, const void *src, size_t bytes, int32_t reps, void *stream, double *ms)
{
    if (!dst || !src || !ms || reps <= 0 || bytes % 16) return fail(WLB_ERR_ARG, "bad copy probe arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(launch_copy(dst, src, bytes, st));
    HIPCHK(hipEventRecord(a, st));
    for (int k = 0; k < reps; ++k) HIPCHK(launch_copy(dst, src, bytes, st));
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, a, b));
    *ms = (double)t / reps;
    hipEventDestroy(a);
    hipEventDestroy(b);
    return WLB_OK;
}

}  // extern "C"
