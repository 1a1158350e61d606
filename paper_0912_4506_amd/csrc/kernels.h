// Internal interface between the host ABI layer (api.cpp) and the device
// kernels (kernels.hip).  Not installed; the public interface is jacobi.h.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#define JAC_MAX_DEPTH_DEV 8

// Compiled block shapes of the temporally blocked kernel:
//   X(id, CI, R, W): lanes hold CI consecutive i cells and R consecutive j rows,
//   W waves are stacked in j, so a workgroup covers (64*CI) x (W*R) cells.
#define JAC_TILE_MENU(X) \
    X(0, 2, 4, 8)        \
    X(1, 1, 8, 8)        \
    X(2, 1, 6, 8)        \
    X(3, 2, 3, 8)        \
    X(4, 1, 4, 8)        \
    X(5, 2, 2, 8)        \
    X(6, 1, 3, 16)       \
    X(7, 1, 4, 16)       \
    X(8, 2, 2, 16)       \
    X(9, 1, 7, 8)        \
    X(10, 1, 5, 12)      \
    X(11, 1, 5, 16)      \
    X(12, 1, 6, 12)

namespace jac {

// MODE_BATCH is MODE_PLAIN with agent-scope output stores (see batched_kernel);
// MODE_COMP reads and writes one array in two frames (see compressed_kernel)
enum { MODE_PLAIN = 0, MODE_RHS = 1, MODE_TRACE = 2, MODE_BATCH = 3, MODE_COMP = 4 };
enum { FACES_SAVE = 0, FACES_ZERO = 1, FACES_CLEAR_SUM = 2, FACES_ACCUM = 3, FACES_FINALIZE = 4 };

struct GridArgs {
    int64_t nx, ny, nz, sy, sz;
};

// Threads per block of the plain sweep for an interior width nx (its strips
// are 2 * threads cells wide).
int plain_threads(int64_t nx);

struct PlainArgs {
    int nx, ny, nz, kchunk;
    int64_t sy, sz;
};

// Byte offset the blocked kernels give a masked-off output store; planes
// must be smaller (the host refuses planes of this many bytes or more).
constexpr int kDropOffset = 0x7ffffff0;

template <typename real>
struct TbArgs {
    const real *src;
    real *dst;
    const real *rhs;
    real *trace;
    int64_t sy, sz;
    int nx, ny, nz;
    int nti, ntj;       // block columns along i and j
    int hi;             // i-halo (>= depth; even when CI is even, for alignment)
    int64_t fstride;    // MODE_TRACE: values per level of the face trace
    int kchunk;         // output planes per workgroup along k
    // MODE_COMP only: copies of the planes around the k chunk boundaries
    // (2*shift+1 planes per inner boundary, addressed like src), one progress
    // counter per block, the ticket counter, the error flag, the frame shift,
    // the direction of the block order (+1: blocks wait on lower neighbours,
    // -1: on upper ones) and the polls before a wait gives up
    const real *snap;
    int *prog;
    int *ticket;
    int *error;
    int shift, dir, spin_limit;
};

// A compiled kernel instance: entry point, dynamic LDS bytes, threads per block.
struct KernInfo {
    const void *fn;
    size_t lds;
    int threads;
};

// Instances of the temporally blocked pass per mode and dtype (tb_*.hip).
KernInfo tb_info_plain_f64(int cfg, int depth);
KernInfo tb_info_plain_f32(int cfg, int depth);
KernInfo tb_info_rhs_f64(int cfg, int depth);
KernInfo tb_info_rhs_f32(int cfg, int depth);
KernInfo tb_info_trace_f64(int cfg, int depth);
KernInfo tb_info_trace_f32(int cfg, int depth);
KernInfo tb_info_comp_f64(int cfg, int depth);
KernInfo tb_info_comp_f32(int cfg, int depth);

// ------------------------------------------------------------- batched runs --
// Plan image of a batched run (built on the host, uploaded by the caller):
// [BatchHeader][BatchGrid x n][BatchItem x nitems][int pass_start x (maxpasses+1)]
constexpr uint32_t BATCH_MAGIC = 0x4a414342u;  // "JACB"

// order: 0 = items pass by pass (any run mode); 1 = pipelined wavefronts over
// (pass, k chunk), relaxed mode only.
struct BatchHeader {
    uint32_t magic;
    int dtype, n, nitems, ntiles, cfg, t, maxpasses, order, team;
    int64_t grids_off, items_off, pass_off, total_bytes, max_shell;
};

struct BatchGrid {
    const void *a;
    void *b;
    int64_t sy, sz;
    int nx, ny, nz;
    int nti, ntj, nkc, hi, kchunk;
    int T, passes, tiles, counter_off;
    // pipelined runs (relaxed synchronisation, Eq. 3): passes per segment
    // (0: not pipelined), lower and upper distances and team delay in k
    // chunks beyond the one-chunk halo (du = 0: no upper bound)
    int team, dl, du, dt;
};

// One block of one pass of one grid.  Items are ordered pass by pass, or in
// pipeline wavefronts; in either order every block an item waits on comes
// earlier.  delay: sleep rounds (s_sleep 127, about 3.4 us each) before the
// item starts; 0 except in stress runs of the relaxed synchronisation.
struct BatchItem {
    int grid, pass, tile, delay;
};

// Persistent (relaxed) mode: blocks pop items in order and wait for the
// neighbouring blocks of the previous pass through per-block counters.
// Lockstep mode: one launch per pass, one item per workgroup.
// fixed = 1: the instance for launches whose items all have depth `depth`
KernInfo batch_info_f64(int cfg, int depth, int fixed);
KernInfo batch_info_f32(int cfg, int depth, int fixed);

struct BatchLaunch {
    const BatchGrid *grids;
    const BatchItem *items;
    int begin, end;      // item range of this launch
    int *counters;       // [0] next item, [1 + c] pass counter of block c
    int *error;          // set to 1 when a wait gives up
    int persistent;
    int spin_limit;      // polls before a wait gives up
};

struct TileShape {
    int id, ci, rows, waves;
    int bx() const { return 64 * ci; }
    int by() const { return rows * waves; }
};

template <typename real>
hipError_t launch_plain(const real *a, real *b, const PlainArgs &p, hipStream_t st);
template <typename real>
hipError_t launch_tblock(int cfg, int depth, int mode, const TbArgs<real> &p, int nblocks,
                         hipStream_t st);
template <typename real>
hipError_t launch_copy_shell(const real *a, real *b, const GridArgs &g, hipStream_t st);
// Shell copy a -> b of every grid of a batch, and a counter reset (n ints = 0).
template <typename real>
hipError_t launch_batch_shells(const BatchGrid *grids, int n, int64_t max_shell, hipStream_t st);
hipError_t launch_zero_ints(int *x, int64_t n, hipStream_t st);
// The whole shell of a grid, edges and corners included, to (save = 1) or
// from (save = 0) a compact array of shell_count(g) values.
int64_t shell_count(const GridArgs &g);
template <typename real>
hipError_t launch_shell_store(int save, real *grid, real *store, const GridArgs &g, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);
// Shell-face helpers of the adjoint (FACES_*): save grid faces into G, zero
// the grid's faces, clear S, accumulate S += trace levels in order, or write
// grid faces = G + S/6.
template <typename real>
hipError_t launch_faces(int op, real *grid, real *G, real *S, const real *tr, const GridArgs &g,
                        int64_t F, int depth, hipStream_t st);

// Refinement helpers: FP64 residual (r32 = (float)r, norm2 = |r|^2
// through residual_partials(g) per-block partial sums), x += e32, and the
// fused form: xnew = x + e32, the residual of xnew, z = 0 (interiors).
int64_t residual_partials(const GridArgs &g);
hipError_t launch_residual(const double *x, float *r32, double *partial, double *norm2,
                           const GridArgs &g, hipStream_t st);
hipError_t launch_update_residual(const double *x, const float *e32, double *xnew, float *z,
                                  float *r32, double *partial, double *norm2, const GridArgs &g,
                                  hipStream_t st);
// The allocation-free residual: partial sums go to a fixed device array
// (noalloc_partials_max() doubles per GPU); noalloc_scratch gives its device
// address for the current device; residual_partials_plain(g) is how many
// partial sums launch_residual writes for grid g.
int64_t noalloc_partials_max();
int64_t residual_partials_plain(const GridArgs &g);
hipError_t noalloc_scratch(double **out);
template <typename real>
hipError_t launch_grid_fill(real *x, real v, const GridArgs &g, hipStream_t st);
hipError_t launch_update(double *x, const float *e32, const GridArgs &g, hipStream_t st);
template <typename real>
hipError_t launch_grid_add(real *dst, const real *src, const GridArgs &g, hipStream_t st);

hipError_t launch_batched(int dtype, int cfg, int depth, int fixed, const BatchLaunch &L, int nblocks,
                          hipStream_t st);
int batched_occupancy(int dtype, int cfg, int depth, int fixed);
int batched_scratch(int dtype, int cfg, int depth, int fixed);

// D3Q19 lattice Boltzmann step (lbm.hip): populations of a periodic nx x ny x
// nz box, 19 arrays of n = nx*ny*nz values, streamed and collided from f
// into out.
struct LbmArgs {
    int nx, ny, nz;
    int64_t n;
    double omega;
};
template <typename real>
hipError_t launch_lbm_d3q19(const real *f, real *out, const LbmArgs &p, hipStream_t st);
// Two steps in one pass (temporal blocking at depth 2): z chunks of `kchunk`
// output planes per workgroup.
template <typename real>
hipError_t launch_lbm_d3q19_x2(const real *f, real *out, const LbmArgs &p, int kchunk,
                               hipStream_t st);
// Shape of the depth-2 pass: the workgroup's level-1 region (x by y cells,
// one per thread) and the output tile inside it (one cell less per side);
// measured at 256^3: 32 x 8 in FP64 (two workgroups per CU fit the LDS),
// 32 x 16 in FP32.
constexpr int lbm2_region_x(size_t) { return 32; }
constexpr int lbm2_region_y(size_t elem) { return elem == 8 ? 8 : 16; }

// Per-lane scratch (register spill) bytes of a tblock instance, -1 if none.
int tblock_scratch(int dtype, int cfg, int depth, int mode);

// Resident workgroups per CU of a tblock instance (0 when it cannot launch).
int tblock_occupancy(int dtype, int cfg, int depth, int mode);

}  // namespace jac
