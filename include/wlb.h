/*
 * wlb.h -- C ABI of the MI355X lattice Boltzmann library (libwlb.so).
 *
 * The library advances the lattice Boltzmann method over a list of
 * structured blocks on one GPU, following Bauer et al., "waLBerla: A
 * block-structured high-performance framework for multiphysics simulations":
 *   - blocks are containers of uniformly gridded cells with one ghost layer
 *     (Sec. 3.1 and Sec. 4.1);
 *   - a sweep (kernel) runs on every block, then a ghost-layer exchange
 *     between neighbouring blocks makes the state consistent (Sec. 4.2);
 *     between blocks on the same device the exchange is a direct copy
 *     without buffers (Sec. 3.3);
 *   - the sweep is the fused collide-and-stream update of Eq. 2 with the
 *     moments of Eq. 1 and the MRT operator of Eq. 3 (SRT and TRT as special
 *     relaxation matrices), a relaxation time that may vary per cell from a
 *     closure, bounce-back / pressure boundaries and a body force
 *     (Sec. 5.1.1);
 *   - initial data and results live in host arrays that are copied to and
 *     from the device only at set-up and after many steps (Sec. 4.3).
 *
 * Conventions
 *   Velocity sets (Sec. 5.1.1 names all four): D2Q9, D3Q15, D3Q19, D3Q27.
 *     D3Q27 population order: 0 rest; 1..6 (+-1,0,0), (0,+-1,0), (0,0,+-1);
 *     7..18 the edges (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1),
 *     (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1),
 *     (0,-1,1); 19..26 the corners (1,1,1), (-1,-1,-1), (1,1,-1),
 *     (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1).  D3Q19 is
 *     populations 0..18 of that order; D3Q15 is 0..6 followed by the eight
 *     corners 19..26; D2Q9 is 0..4 followed by the xy edges 7..10 (every
 *     z component 0: each z plane is an independent 2D lattice).  In every
 *     set the opposite of an odd population i is i+1.  Weights by |c|^2:
 *     D2Q9 4/9, 1/9, 1/36; D3Q15 2/9, 1/9, 1/72; D3Q19 1/3, 1/18, 1/36;
 *     D3Q27 8/27, 2/27, 1/54, 1/216; c_s^2 = 1/3.  MRT needs D3Q19 or
 *     D3Q27, KBC and the cumulant collision D3Q27.
 *   State: populations are stored as deviations d_i = f_i - w_i.
 *   Global host arrays cover the bounding box `domain` with x fastest,
 *     then y, then z: scalar fields [N], vector fields [3][N] (component
 *     major), population fields [q][N], N = domain[0]*domain[1]*domain[2].
 *   Status: every int-returning call returns WLB_OK (0) or a negative
 *     WLB_ERR_* code; wlb_last_error() then describes the failure (per
 *     thread).  No C++ exception crosses the ABI.
 *   Ownership: host arrays belong to the caller and are only read or written
 *     during the call.  Device memory is one arena that the caller allocates
 *     (size from wlb_blocks_create) and binds; the library never allocates
 *     or frees device memory.  The handle owns host-side descriptors, the
 *     captured HIP graph and the tuning state.
 *   Streams: all device work is enqueued on the stream given to
 *     wlb_blocks_bind.  Calls that return host data synchronise that stream.
 *     A handle must not be used from two threads at once.
 */
#ifndef WLB_H
#define WLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WLB_OK 0
#define WLB_ERR_ARG (-1)         /* bad sizes, blocks that do not tile the domain, tau <= 1/2, ... */
#define WLB_ERR_HIP (-2)         /* a HIP runtime call failed */
#define WLB_ERR_STATE (-3)       /* call out of order (e.g. step before bind/init) */
#define WLB_ERR_DIVERGED (-4)    /* health check: non-finite mass or max|u| above the limit */
#define WLB_ERR_UNSUPPORTED (-5) /* combination not implemented */

enum { WLB_D2Q9 = 9, WLB_D3Q15 = 15, WLB_D3Q19 = 19, WLB_D3Q27 = 27 };
/* SRT, TRT, MRT (Eq. 3); KBC: the MRT basis with the entropic choice of the
 * trace and higher-order rates per cell (Sec. 5.1.1, Boesch, Chikatamarla,
 * Karlin 2015; D3Q27 only; omega_bulk / omega_higher unused); CUMULANT:
 * second-order cumulants relaxed with 1/tau (deviatoric) and omega_bulk
 * (trace), all higher cumulants with rate 1 (Sec. 5.1.1, Geier et al. 2015;
 * D3Q27 only; omega_higher unused). */
enum { WLB_SRT = 0, WLB_TRT = 1, WLB_MRT = 2, WLB_KBC = 3, WLB_CUMULANT = 4 };
/* storage type of the deviations; collision runs in FP64 for WLB_F64 and in
 * FP32 otherwise; conversions round to nearest even, no denormal flush */
enum { WLB_F64 = 0, WLB_F32 = 1, WLB_F16DEV = 2, WLB_BF16DEV = 3 };
enum { WLB_CLOSURE_NONE = 0, WLB_CLOSURE_SMAG = 1, WLB_CLOSURE_MLP = 2 };

/* Number of float parameters of the MLP closure (7 -> 32 -> 32 -> 1), packed
 * as mean[7], inv_std[7], W1[32][7], b1[32], W2[32][32], b2[32], w3[32], b3
 * (row = output unit, column = input). */
#define WLB_MLP_NPARAM 1359

typedef struct wlb_blocks *wlb_blocks_t;

/* One block: global cell coordinates of its first interior cell and its
 * interior extent.  Blocks must tile the domain exactly and neighbours must
 * share whole faces (a rectilinear block grid). */
typedef struct {
    int32_t origin[3];
    int32_t size[3];
} wlb_block_desc;

/* Parameters of the update (Sec. 5.1.1).
 *   tau          shear relaxation time tau_0 (> 1/2)
 *   magic        TRT parameter Lambda = (tau+ - 1/2)(tau- - 1/2)
 *   omega_bulk   MRT rate of the trace moment x2+y2+z2
 *   omega_higher MRT rate of all moments of order >= 3
 *   force        body force density (Guo forcing); u = (sum c d + F/2)/rho
 *   closure      WLB_CLOSURE_*: per-cell tau from the non-equilibrium stress
 *   cs_smag      Smagorinsky constant C_s (closure SMAG, and MLP fallback)
 *   mlp          host pointer to WLB_MLP_NPARAM floats (closure MLP), copied
 *   pressure_axis  -1, or the non-periodic axis whose two faces carry the
 *                density rho_in (low end) / rho_out (high end) through
 *                anti-bounce-back; other non-periodic faces are half-way
 *                bounce-back walls
 *   health_every check mass and max|u| every this many steps (0 = never);
 *                a failed check makes wlb_lbm_step return WLB_ERR_DIVERGED
 *   health_umax  limit on max|u| for the health check (<= 0 means 0.3)
 *   autotune     1: time candidate tile shapes and launch sizes at init and
 *                keep the fastest; 0: default shapes */
typedef struct {
    double tau;
    double magic;
    double omega_bulk;
    double omega_higher;
    double force[3];
    int32_t closure;
    double cs_smag;
    const float *mlp;
    int32_t pressure_axis;
    double rho_in;
    double rho_out;
    int32_t health_every;
    double health_umax;
    int32_t autotune;
} wlb_lbm_params;

/* Create a block set (Sec. 3.1: the domain split into blocks that are the
 * containers of the simulation data; Sec. 4.1: each block a uniform grid of
 * cells with ghost layers, translating between block-local and global cell
 * coordinates).  d[n] describes the blocks, domain[3] the bounding box,
 * periodic[3] which axes wrap.  stencil = WLB_D2Q9/D3Q15/D3Q19/D3Q27, storage =
 * WLB_F64/F32/F16DEV/BF16DEV.  Builds the 26-neighbour table (periodic links
 * included), the tile list and the exchange work list, and returns in
 * *arena_bytes the size of the device arena to bind.
 * Errors: WLB_ERR_ARG for empty/oversized blocks, overlapping blocks, blocks
 * that do not cover the domain, or neighbours that do not share whole faces. */
int wlb_blocks_create(const wlb_block_desc *d, int32_t n, const int32_t domain[3], const int32_t periodic[3],
                      int32_t stencil, int32_t storage, size_t *arena_bytes, wlb_blocks_t *out);

/* Bind a caller-owned device arena (>= arena_bytes, 256-byte aligned) and the
 * HIP stream (a hipStream_t; must not be the null stream) on which all work
 * of this handle runs (Sec. 4.3: the GPU fields, laid out with padding so
 * that rows are aligned, Sec. 4.2).  Uploads the descriptor tables.  The arena must stay
 * allocated until wlb_blocks_destroy. */
int wlb_blocks_bind(wlb_blocks_t h, void *device_arena, size_t bytes, void *hip_stream);

/* Initialise the populations to the equilibrium of rho[N], u[3][N] (host,
 * FP64, global order) and the geometry from solid[N] (host, 1 = solid, may be
 * NULL for no solid cells).  Sec. 4.3: the initial state is set up in host
 * (mirror) arrays and transferred to the GPU once; Sec. 4.4: the geometry
 * becomes per-cell flags that select the boundary treatment.  collision = WLB_SRT/TRT/MRT/KBC/CUMULANT.  Resets the step
 * counter.  Runs the tile autotuner when p->autotune is set (the state is
 * re-initialised afterwards).  Synchronises the stream.
 * Errors: WLB_ERR_ARG (tau <= 1/2, bad pressure axis, MLP without weights),
 * WLB_ERR_STATE (not bound), WLB_ERR_UNSUPPORTED (MRT, KBC or the cumulant
 * collision with the MLP closure; MRT without D3Q19 / D3Q27; KBC or the
 * cumulant collision without D3Q27; the MLP closure without D3Q19). */
int wlb_lbm_init(wlb_blocks_t h, int32_t collision, const wlb_lbm_params *p, const double *rho, const double *u,
                 const uint8_t *solid);

/* Advance nsteps time steps, each one sweep (collide + stream, Eq. 2)
 * followed by the ghost-layer exchange.  Asynchronous on the bound stream
 * unless a health check falls in the range (then it synchronises). */
int wlb_lbm_step(wlb_blocks_t h, int32_t nsteps);

/* One sweep over all blocks without the following exchange (the sweep of
 * Sec. 4.2 on its own).  Must be followed by wlb_ghost_exchange before the
 * next sweep; wlb_lbm_step(h, 1) == wlb_lbm_sweep + wlb_ghost_exchange. */
int wlb_lbm_sweep(wlb_blocks_t h);

/* Ghost-layer exchange between the blocks (Sec. 4.1 and Sec. 4.2: after a
 * sweep the ghost layers propagate the updated data to neighbouring blocks;
 * Sec. 3.3: between blocks of one process a direct copy without buffers).
 * Exchange the ghost layers that the last sweep requires (after an even sweep
 * the neighbours' outgoing populations are copied into the ghost layer;
 * after an odd sweep the populations written into the ghost layer are
 * copied into the neighbours).  Idempotent; asynchronous. */
int wlb_ghost_exchange(wlb_blocks_t h);

/* Moments (Eq. 1) of the current state: rho[N] and u[3][N] (host, may be
 * NULL to skip), u = (sum c d + F/2)/rho; solid cells get rho = 0, u = 0.
 * totals[8] (may be NULL) = mass, momentum x/y/z (sum rho u), kinetic energy
 * sum rho|u|^2/2, max|u|, number of fluid cells, steps taken.  Reductions in
 * FP64 with a fixed order (deterministic).  Synchronises the stream. */
int wlb_moments_get(wlb_blocks_t h, double *rho, double *u, double totals[8]);

/* Force handed to the obstacles during the last step by momentum exchange
 * (section "Geometrically fully resolved simulations": the momentum-exchange
 * method of Ladd and Aidun et al.).  Every post-collision population f*_i of
 * a fluid cell whose target x + c_i is a solid cell or lies beyond a wall
 * (half-way bounce-back) delivers 2 c_i f*_i; links through pressure faces
 * do not count.  out[8] (host, caller-owned) = force on the solid cells
 * x/y/z, force on the walls x/y/z, number of solid links, number of wall
 * links, in lattice units (mass = density x cells, per step).  Reads only
 * the bounce-back populations of the current state (no exchange needed);
 * FP64 sums in a fixed order; synchronises the stream.
 * Errors: WLB_ERR_ARG (null argument), WLB_ERR_STATE (before wlb_lbm_init,
 * or no step since it), WLB_ERR_HIP. */
int wlb_force_get(wlb_blocks_t h, double out[8]);

/* Debug check of the AA pattern's race freedom (Sec. 5.1.1 update rule, in
 * place): every (cell, population slot) must be written by exactly one
 * thread per sweep.  Zeroes the populations and runs one sweep of the given
 * parity (odd = 0: even sweep and the exchange after it; odd = 1: odd sweep
 * and the exchange after it) with the handle's tiles, grid and overlap
 * setting, in kernels where each population store adds 1 to a counter in
 * its place and each exchange copy adds the ghost cell's counter to its
 * target.  counts[q][N] (host, caller-owned, global order, storage slots)
 * receives the counters of every interior (cell, slot): a correct sweep
 * leaves 1 in every slot of a fluid cell and 0 in solid cells.  Needs FP32
 * storage (the counters use its 4-byte slots).  Leaves counters in place of
 * the state: call wlb_lbm_init before the next step.  Synchronises the stream.
 * Errors: WLB_ERR_ARG, WLB_ERR_STATE (before wlb_lbm_init),
 * WLB_ERR_UNSUPPORTED (storage other than FP32), WLB_ERR_HIP. */
int wlb_debug_write_coverage(wlb_blocks_t h, int32_t odd, uint32_t *counts);

/* Population deviations d_i = f_i - w_i of the current state in natural
 * layout d[q][N] (FP64, host), and the reverse (Sec. 3.4: the block data is
 * serialised for checkpoints and restored on restart; Sec. 4.3: results are
 * copied back to host arrays).  set also re-establishes the
 * natural layout so the next sweep is even; solid cells are ignored.  Used
 * for checkpoint / resume (bitwise for every storage type). */
int wlb_pdfs_get(wlb_blocks_t h, double *d);
int wlb_pdfs_set(wlb_blocks_t h, const double *d);

/* Information and tuning. */
typedef struct {
    int64_t steps;          /* steps taken since init */
    int32_t parity;         /* 0: natural layout (next sweep even); 1: swapped */
    int32_t n_blocks;
    int64_t n_cells;        /* interior cells of all blocks */
    int64_t n_fluid;        /* fluid cells */
    int32_t n_tiles;
    int32_t tile[3];        /* tile shape target in use (x, y, z); -1, 0, 0: fluid-cell lists */
    int32_t grid;           /* workgroups per sweep launch (0 = one per tile, -1 = one per tile
                               with XCD-contiguous tile ranges) */
    int32_t lds_staging;    /* odd-sweep kernel in use: 0 direct, 1 LDS-staged, 2 row vectors */
    int32_t n_xchg_items;   /* exchange work items per exchange */
    int64_t xchg_elems;     /* populations copied per exchange */
    size_t arena_bytes;
    size_t pop_bytes;       /* bytes of population storage incl. ghosts */
    int32_t overlap;        /* 1: sweeps split into interior and frontier, exchange overlapped */
    int32_t nt_even;        /* 1: the even sweep's population accesses are non-temporal */
    int32_t nt_odd;         /* 1: the odd sweep's population accesses are non-temporal; 2: only
                               its aligned ones (populations with c_x = 0) */
    int32_t n_class_tiles;  /* classes of x-runs (by y extent) whose tile shape the autotuner
                               set apart from `tile` (0: one shape for every run) */
    int32_t slot_round_kib; /* population slots of 64 MiB or more start on multiples of this
                               many KiB (0: 256-byte alignment only); chosen by the autotuner,
                               16384 otherwise */
} wlb_info_t;
int wlb_info(wlb_blocks_t h, wlb_info_t *out);

/* Use tile shape (tx, ty, tz) (tx*ty*tz <= 256) and `grid` workgroups per
 * sweep launch from now on: 0 = one workgroup per tile (workgroups reach the
 * 8 XCDs round-robin); -1 = one workgroup per tile, the workgroups of each
 * XCD taking one contiguous range of tiles (and of exchange items), so that
 * neighbouring tiles share an L2; > 0 = a persistent grid of that many
 * workgroups looping over the tiles.  tx = 0 packs whole x rows; tx = -1
 * makes the sweeps run over lists of up to 256 fluid cells of one block
 * (no lanes on solid cells; needs a preceding wlb_lbm_init with solid cells
 * and blocks of at most 1024 x 1024 x 4096 cells), all other passes over
 * whole-row tiles.
 * The shape applies to every x-run (it replaces per-class shapes that the
 * autotuner may have chosen).
 * Errors: WLB_ERR_ARG (shape above 256 cells, grid < -1, more tiles than the
 * arena's tile table holds), WLB_ERR_STATE (tx = -1 without fluid lists). */
int wlb_set_tiles(wlb_blocks_t h, int32_t tx, int32_t ty, int32_t tz, int32_t grid);

/* Tile shape of one class of x-runs (Sec. 4.1: blocks of different sizes in
 * one launch): every x-run whose y extent is `y_extent` gets box tiles of
 * (tx, ty, tz) (tx = 0: whole rows), the others keep theirs; the grid and
 * the odd-sweep choice stay.  The autotuner makes the same per-class choice.
 * Results do not depend on it.
 * Errors: WLB_ERR_ARG (null handle, shape above 256 cells or negative, no
 * x-run of that y extent, more tiles than the tile table holds),
 * WLB_ERR_STATE (fluid-cell list tiles in use). */
int wlb_set_class_tiles(wlb_blocks_t h, int32_t y_extent, int32_t tx, int32_t ty, int32_t tz);

/* Slot stride of the population storage (Sec. 4.2: the layout of the
 * fields): slots of 64 MiB or more start on multiples of `kib` KiB (16384,
 * 2048, or 0 = 256-byte alignment only); smaller slots are only aligned.
 * The arena is sized for 16384, the default.  Call after wlb_blocks_bind and
 * before wlb_lbm_init; an init with the autotuner chooses the stride again.
 * Results do not depend on it.
 * Errors: WLB_ERR_ARG (null handle, another value), WLB_ERR_STATE (the
 * populations are already initialised). */
int wlb_set_slot_round(wlb_blocks_t h, int32_t kib);

/* Odd-sweep kernel (Eq. 2 and the AA scheme of Sec. 4.1 are the same in all
 * three; results are bitwise identical):
 *   0 (default) direct: every lane reads and writes its cell's x-shifted
 *     populations one element off the row alignment;
 *   1 LDS staging: the x-shifted populations pass through LDS row buffers
 *     so that all global accesses are row-aligned.  Tiles that are whole
 *     rows of a block wrapping onto itself along x shift around the row
 *     buffer; other row segments load one halo element per row end and
 *     store one element past it, through the block's other end, its ghost
 *     column or an x-neighbour block.  Skipped automatically with
 *     fluid-cell list tiles and when the buffers exceed 64 KiB per
 *     workgroup;
 *   2 row vectors: whole rows, 16 / (element bytes) consecutive cells per
 *     lane, every access one aligned 16-byte vector, the one-cell x shift
 *     done by moving elements between lanes (the lane at a wavefront edge
 *     reads or writes the element crossing it).  Needs every block to wrap
 *     onto itself along x, to hold no solid cells nearby, to have rows that
 *     split into whole vectors of at most 256 lanes, no MLP closure and no
 *     interior/frontier overlap; otherwise the direct sweep runs.
 * wlb_info_t.lds_staging reports the kernel in use.  The autotuner tries all
 * three.
 * Errors: WLB_ERR_ARG for a null handle or a mode outside 0..2. */
int wlb_set_lds_staging(wlb_blocks_t h, int32_t on);

/* Interior/frontier overlap (1) or not (0, default).  Sec. 3.3 and 6: the
 * paper hides communication behind computation; here each sweep is split
 * into the cells at least two rows from every y/z block face that has a
 * neighbour (interior) and the rest (frontier), and in wlb_lbm_step the
 * frontier part and the ghost exchange run on a second HIP stream (created
 * by the library, default priority) while the interior part runs on the
 * bound stream; each step joins both.  Results are bitwise identical to the
 * sequential order.  With per-kernel timing on, or through wlb_lbm_sweep /
 * wlb_ghost_exchange, the parts run in turn on the bound stream.  The
 * autotuner tries it for the best tile configuration when blocks exchange.
 * Errors: WLB_ERR_ARG (null handle), WLB_ERR_HIP (stream creation). */
int wlb_set_overlap(wlb_blocks_t h, int32_t on);

/* Non-temporal hint (1, default) or ordinary cached accesses (0) for the
 * population loads and stores of the even and of the odd sweep; for the odd
 * sweep also 2: the hint on its aligned accesses only (the populations with
 * c_x = 0, whole lines per wavefront), the others cached.  Streamed once per
 * sweep, the populations usually gain from the hint; accesses one element
 * off the row alignment, and short rows whose cache lines neighbouring waves
 * share, can gain from the cache instead.  Results are bitwise identical
 * either way.  The autotuner tries all six settings (with and without LDS
 * staging; 2 and 1 are the same for the LDS-staged and row-vector odd
 * sweeps, whose accesses are all aligned) for the best tile configuration.
 * Errors: WLB_ERR_ARG for a null handle or an odd-sweep hint outside 0..2. */
int wlb_set_nontemporal(wlb_blocks_t h, int32_t even, int32_t odd);

/* Use (1) or bypass (0) the captured HIP graph in wlb_lbm_step. */
int wlb_set_graph(wlb_blocks_t h, int32_t on);

/* Per-kernel timing: when on, wlb_lbm_step launches eagerly and brackets
 * every kernel with HIP events on the bound stream; wlb_kernel_times then
 * returns the summed milliseconds and launch counts of [even sweep, odd
 * sweep, exchange after even, exchange after odd] since the last reset
 * (synchronises).  Turning it on resets the sums. */
int wlb_set_kernel_timing(wlb_blocks_t h, int32_t on);
int wlb_kernel_times(wlb_blocks_t h, double ms[4], int64_t launches[4]);

/* --- learned closure: network evaluation and training ------------------ */

/* Box filter of the current state for LES training data: for every coarse
 * cell of a factor^3 coarsening, the averages of rho, u (Guo velocity) and
 * u_a u_b over its fine cells, into out[10][Nc] (device, FP64, coarse cells
 * in global order; channels rho, ux, uy, uz, uxux, uyuy, uzuz, uxuy, uxuz,
 * uyuz).  Single-block handles whose domain the factor divides.
 * Synchronises the bound stream.  (Sec. 4.4: data gathered for evaluation.) */
int wlb_box_filter(wlb_blocks_t h, int32_t factor, double *out);

/* Training pairs of the learned closure from filtered fields filt[10][Nc]
 * (device, the layout of wlb_box_filter) on a periodic coarse grid nc[3]:
 * target[Nc] = 3 nu_t with nu_t = max(0, -dev(tau_sgs) : S / (2 S : S)),
 * tau_sgs = avg(u u) - u u, S = symmetric central-difference gradient of the
 * filtered u; raw[Nc][7] = (Pi = -(2/3) rho (tau0 + target) S (xx, yy, zz,
 * xy, xz, yz), rho - 1).  Device pointers; asynchronous on `hip_stream`. */
int wlb_les_targets(const double *filt, const int32_t nc[3], double tau0, float *raw, float *target,
                    void *hip_stream);

/* Bytes of device workspace wlb_mlp_forward needs. */
#define WLB_MLP_WORKSPACE 4096

/* Evaluate the closure network (7 -> 32 -> 32 -> 1, see WLB_MLP_NPARAM) with
 * the same matrix-core code the sweep uses: raw[n][7] (device, FP32: Pi_xx,
 * Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz, rho - 1) -> out[n] (device, output o;
 * tau = tau0 + softplus(o)) and fallback[n] (device, 1 where a standardised
 * feature exceeds 8 in magnitude or o is not finite: the sweep then uses the
 * Smagorinsky time).  params: host, WLB_MLP_NPARAM floats.  workspace:
 * device, WLB_MLP_WORKSPACE bytes, 16-byte aligned.  Synchronises `hip_stream`.
 * (Paper Sec. 5.1.1: relaxation times that vary per cell.) */
int wlb_mlp_forward(const float *params, void *workspace, const float *raw, int64_t n, float *out, int32_t *fallback,
                    void *hip_stream);

/* Device workspace bytes wlb_mlp_grad needs for a minibatch of n samples. */
size_t wlb_mlp_grad_workspace(int64_t n);

/* Gradient of L = (1/n) sum ((softplus(o_s) - target_s) * inv_scale)^2 with
 * respect to all parameters (zero for mean / inv_std), FP32, deterministic.
 * params, raw[n][7], target[n], grad[WLB_MLP_NPARAM], loss[1], workspace:
 * device pointers.  Asynchronous on `hip_stream`. */
int wlb_mlp_grad(const float *params, const float *raw, const float *target, int64_t n, double inv_scale, float *grad,
                 float *loss, void *workspace, size_t ws_bytes, void *hip_stream);

/* Largest minibatch of wlb_mlp_grad_noalloc. */
#define WLB_MLP_NOALLOC_MAX_SAMPLES 262144

/* wlb_mlp_grad without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results (bit for bit) as wlb_mlp_grad; the per-workgroup partial sums go to
 * a fixed library-owned device array of WLB_MLP_NOALLOC_MAX_SAMPLES / 256 x
 * (WLB_MLP_NPARAM + 1) floats (5.6 MB), one per GPU, held until the process
 * ends.  The call allocates nothing.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  Asynchronous on
 * `hip_stream` (the device current at the call must be the stream's).
 * Errors: WLB_ERR_ARG (null argument, n <= 0, n > WLB_MLP_NOALLOC_MAX_SAMPLES),
 * WLB_ERR_HIP. */
int wlb_mlp_grad_noalloc(const float *params, const float *raw, const float *target, int64_t n, double inv_scale,
                         float *grad, float *loss, void *hip_stream);

/* One Adam update of the FP32 master parameters in place (mean / inv_std
 * untouched); m, v: device moment buffers (WLB_MLP_NPARAM floats, zero at
 * step 1); step counts from 1.  Asynchronous on `hip_stream`. */
int wlb_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr, double beta1,
                 double beta2, double eps, void *hip_stream);

/* Release the handle (not the arena). */
void wlb_blocks_destroy(wlb_blocks_t h);

const char *wlb_last_error(void);

/* Achievable device bandwidth probe: copy `bytes` (multiple of 16) from src
 * to dst (device pointers) `reps` times on `hip_stream` with the library's
 * own copy kernel; returns the mean milliseconds per copy in *ms. */
int wlb_copy_probe(void *dst, const void *src, size_t bytes, int32_t reps, void *hip_stream, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* WLB_H */
