/*
 * jacobi.h -- C ABI of the MI355X (gfx950) Jacobi library, libjacobi.so.
 *
 * The method: repeated sweeps of the 3D Jacobi update (update equation of
 * Sect. 1.1 of Wittmann, Hager, Wellein, "Multicore-aware parallel temporal
 * blocking of stencil codes for shared and distributed memory"):
 *     B(i,j,k) = ( A(i-1,j,k) + A(i+1,j,k) + A(i,j-1,k) + A(i,j+1,k)
 *                + A(i,j,k-1) + A(i,j,k+1) ) / 6
 * over the interior of a grid whose one-cell shell holds fixed Dirichlet data,
 * writing grids A and B in turn (same section).  Temporal blocking (the idea
 * of Sect. 1.1, the shrinking-overlap rule of Sect. 2.1) fuses t sweeps into
 * one pass over device memory.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Buffers are DEVICE pointers owned by the caller.  The library never
 *    allocates, frees or retains them.  Host pointers are named as such.
 *  - Element (i,j,k), 0 <= i <= nx+1, 0 <= j <= ny+1, 0 <= k <= nz+1, of a grid
 *    lives at base[i + j*sy + k*sz]: i is contiguous.  Index 0 and n+1 on any
 *    axis is the Dirichlet shell, which no call writes (except where stated).
 *    Only the six face layers of the shell are ever read; the 12 edges and 8
 *    corners of the shell are never read.
 *  - dtype: JAC_F32 (float) or JAC_F64 (double); all grids of a call share it.
 *  - Arithmetic: FP64 sums the six neighbours left to right in the printed
 *    order (i-1, i+1, j-1, j+1, k-1, k+1) and divides by 6.  jacobi_plain and
 *    the adjoint's shell-face gradient divide exactly as IEEE division does,
 *    for every input (infinities, NaN, subnormals and signed zeros included).
 *    The temporally blocked passes (jacobi_tblock, the adjoint's interior,
 *    batched, pipelined and compressed runs) divide in three operations whose
 *    result is the IEEE quotient whenever that quotient is zero (of either
 *    sign) or a normal number: so wherever every sum is finite and every
 *    nonzero quotient is at least 2^-1022 in magnitude, each FP64 result is
 *    bitwise the plain sequential result, whatever the blocking depth, tile
 *    or pass split.  Outside that range the blocked passes differ from IEEE
 *    division in two ways only: a sum of +-Inf gives NaN instead of +-Inf
 *    (so the cells that the oracle makes infinite hold NaN or the same
 *    infinity, and every finite cell is bitwise), and a quotient in the
 *    subnormal range may be one subnormal step (2^-1074) off, a difference
 *    later levels carry along (at most about 2 steps per level).  (Checking
 *    every quotient costs one more vector instruction per cell and level in
 *    the blocked pass, about 7% more, and the branch to redo it registers.)
 *    FP32 sums in the same order and multiplies by the float nearest 1/6.
 *  - Calls enqueue work on `stream` (a hipStream_t; NULL = the null stream)
 *    and return without synchronising.  Argument checks happen before any
 *    HIP call and are synchronous: a failed check returns JAC_EARG and
 *    enqueues nothing.  JAC_EHIP reports an error the HIP runtime returned
 *    while enqueuing; faults inside kernels surface at the caller's next
 *    synchronisation.  jacobi_last_error() describes the last failure of the
 *    calling thread.  No exception crosses the ABI.
 *  - Ping-pong results: `a` holds level 0 on entry.  The library copies a's
 *    shell into b (O(N^2) work) and ignores b's other contents.  On return
 *    *out_idx says where the result is: 0 = a, 1 = b.  It equals the number
 *    of passes over memory modulo 2 (one pass per sweep for jacobi_plain,
 *    so there out_idx = T mod 2).  The other buffer holds an intermediate
 *    level.
 *  - Thread safety: calls are independent; concurrent calls on different
 *    buffers are safe.
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JACOBI_ABI_VERSION 3

/* Grid geometry.  nx, ny, nz >= 1 are the interior extents.  sy and sz are the
 * element strides of j and k; 0 selects the dense strides sy = nx+2 and
 * sz = sy*(ny+2).  Non-zero strides must satisfy sy >= nx+2, sz >= sy*(ny+2). */
typedef struct jac_grid {
    int64_t nx, ny, nz;
    int64_t sy, sz;
} jac_grid_t;

/* Blocking parameters of one temporally blocked call.
 *   t      sweeps fused per pass over memory, 1..JAC_MAX_DEPTH (0 = library
 *          choice).  T sweeps take ceil(T/t) passes; the depths of the passes
 *          differ by at most one.
 *   bx, by i- and j-extent of the block of cells one workgroup updates at every
 *          level, recomputed halo included (the valid part shrinks by one
 *          cell per side and level, Sect. 2.1).  Supported pairs are listed by
 *          jacobi_tile_menu(); 0 = library choice.
 *   kchunk planes of output per workgroup along k (the k range is split so
 *          that the chip has enough workgroups); 0 = library choice.
 *   waves  64-lane wavefronts per workgroup for the block (several kernels
 *          may cover one bx x by, e.g. 8 waves of 6 rows or 16 waves of 3);
 *          0 = library choice. */
typedef struct jac_tile {
    int32_t t, bx, by, kchunk, waves;
} jac_tile_t;

#define JAC_MAX_DEPTH 8

enum { JAC_F32 = 0, JAC_F64 = 1 };
enum {
    JAC_OK = 0,
    JAC_EARG = -1,         /* invalid argument (see jacobi_last_error) */
    JAC_EHIP = -2,         /* the HIP runtime returned an error */
    JAC_EWORKSPACE = -3,   /* workspace missing or too small */
    JAC_EUNSUPPORTED = -4  /* valid request the library has no kernel for */
};

/* Library version (JACOBI_ABI_VERSION of the build).  3: adds
 * jacobi_grid_add, jacobi_batched_stress and the jacobi_tune_* calls (and, in
 * lbm.h, lbm_d3q19_blocked); 2: the pipelined plan takes jac_pipeline_t. */
int jacobi_version(void);

/* Description of the last failure on the calling thread ("" if none).  The
 * string stays valid until the thread's next call into the library. */
const char *jacobi_last_error(void);

/* T plain sweeps, one pass over memory per sweep (the standard Jacobi
 * iteration of Sect. 1.1, whose memory-bound rate Eq. 2 models).
 * a: level 0 on entry; b: second grid of the pair.  T >= 0 (T = 0: nothing is
 * enqueued, *out_idx = 0). */
int jacobi_plain(int dtype, const jac_grid_t *g, void *a, void *b, int T,
                 void *stream, int *out_idx);

/* T sweeps fused t at a time (temporal blocking, Sect. 1.1; overlapped tiles
 * whose update s covers a region one layer wider per remaining level,
 * Sect. 2.1).  tile == NULL or zero fields: library choice.
 * rhs == NULL: the update equation of Sect. 1.1.  rhs != NULL: each sweep
 * computes (six neighbours + rhs(i,j,k)) / 6, Jacobi's method for
 * (6I - adjacency) e = rhs; rhs is a grid of the same dtype and geometry
 * (shell ignored), read-only, not overlapping a or b.  The rhs term is added
 * after the six neighbours, so FP64 results stay bitwise those of the plain
 * sequential iteration (within the range stated under Arithmetic above). */
int jacobi_tblock(int dtype, const jac_grid_t *g, void *a, void *b, int T,
                  const jac_tile_t *tile, const void *rhs, void *stream,
                  int *out_idx);

/* Adjoint of T sweeps.  The sweep map is linear: with x the interior and g the
 * shell, x_s = M x_{s-1} + G g with M = (interior adjacency)/6, and the
 * output's shell is g.  On entry lam_a holds dL/d(level T) for the whole
 * array.  On return the buffer named by *out_idx holds dL/d(level 0):
 *   interior:   lambda_0, where lambda_T = interior of the input and
 *               lambda_{s-1} = M lambda_s;
 *   face shell: input(b) + S_b / 6, S_b = lambda_T(in(b)) + ... + lambda_1(in(b))
 *               summed in that order, in(b) the interior neighbour of b;
 *   shell edges and corners: input(b).
 * lam_b: second grid of the pair (contents ignored).  ws: device workspace
 * of at least jacobi_adjoint_workspace(dtype, g, t) bytes (t as in tile,
 * 0 = library choice), aligned to the element size, not overlapping the grids.
 * T = 0 enqueues nothing: the input is the gradient (*out_idx = 0).  T > 0
 * returns JAC_EUNSUPPORTED, before any launch, when one level of face values
 * (2(ny nz + nx nz + nx ny) elements) takes 2 GiB or more. */
/* dst += src on every element of a grid, shell included, one rounding per
 * element.  It is the step between two adjoint segments when a loss also
 * depends on an intermediate level s: the gradient arriving at level s is
 * added to the adjoint of the later levels before the earlier segment runs
 * (the sweep map is linear, so the adjoint of a sum of losses is the sum of
 * their adjoints).  dst and src: grids of the same dtype and geometry,
 * aligned to the element size; they must not overlap unless dst == src. */
int jacobi_grid_add(int dtype, const jac_grid_t *g, void *dst, const void *src,
                    void *stream);

size_t jacobi_adjoint_workspace(int dtype, const jac_grid_t *g, int t);
int jacobi_adjoint(int dtype, const jac_grid_t *g, void *lam_a, void *lam_b,
                   int T, const jac_tile_t *tile, void *ws, size_t ws_bytes,
                   void *stream, int *out_idx);

/* Batched runs: many independent grids (each with its own geometry and
 * sweep count) in one launch.  Two steps, so that the launch needs no host
 * data and can be captured in a hipGraph and replayed:
 *  1. jacobi_batched_plan (host only): lays out a plan image in plan_host
 *     (jacobi_batched_plan_bytes(...) bytes, host memory): per-grid block
 *     geometry and the list of (grid, pass, block) work items in pass order.
 *     g, a, b, T: n-entry host arrays (a[m], b[m] device grids of grid m,
 *     not overlapping each other or any other grid's).  tile: one blocking
 *     choice for the whole batch (NULL or zero fields = library choice).
 *     out_idx_host[m] receives where grid m's result will be (0 = a, 1 = b).
 *  2. The caller copies the image to device memory (plan_dev, 16-byte
 *     aligned), then jacobi_batched_run enqueues: a shell copy a -> b for
 *     every grid, then either
 *       JAC_BATCH_RELAXED: one persistent launch; workgroups take work items
 *         in order and wait, through one counter per block, until the
 *         neighbouring blocks of the same grid finished the previous pass
 *         (the lower-bound condition of the relaxed synchronisation of
 *         Sect. 1.3, Eq. 3, per block instead of per thread), or
 *       JAC_BATCH_LOCKSTEP: one launch per pass (a global barrier between
 *         passes, the scheme relaxed synchronisation replaces).
 *     ws: device workspace of jacobi_batched_workspace(plan_host) bytes
 *     (the counters; reset by the run itself, every run).  Its last int is
 *     an error flag: a relaxed-mode wait that has not ended after about
 *     2^20 polls gives up and sets it to 1, and every workgroup then stops
 *     (results are invalid); the caller may read it after synchronising.  plan_host must be the image
 *     plan_dev was copied from. */
enum { JAC_BATCH_RELAXED = 0, JAC_BATCH_LOCKSTEP = 1 };
size_t jacobi_batched_plan_bytes(int dtype, int n, const jac_grid_t *g,
                                 const int *T, const jac_tile_t *tile);
int jacobi_batched_plan(int dtype, int n, const jac_grid_t *g, void *const *a,
                        void *const *b, const int *T, const jac_tile_t *tile,
                        void *plan_host, size_t plan_bytes, int *out_idx_host);
size_t jacobi_batched_workspace(const void *plan_host);
int jacobi_batched_run(const void *plan_host, const void *plan_dev, void *ws,
                       size_t ws_bytes, int mode, void *stream);

/* Stress form of a plan, for testing the relaxed synchronisation of a
 * batched or pipelined plan (host only, edits plan_host in place, before it
 * is copied to the device).  The items of each pass are shuffled
 * (pass-ordered plans only; a pipelined plan keeps its order), and about a
 * quarter of all items get a start delay of 1..max_delay sleep rounds of
 * about 3.4 us each (max_delay 0..64; 0 = no delays), both drawn from
 * `seed` (splitmix64).  Every item still waits only on items of earlier
 * passes, so the waits still end; a run of the stressed plan must give
 * bitwise the results of the plain one.  plan_bytes: the size of the buffer
 * at plan_host. */
int jacobi_batched_stress(void *plan_host, size_t plan_bytes, unsigned seed,
                          int max_delay);

/* Pipelined temporal blocking of one grid: the team pipeline of Sect. 1.3 with
 * the relaxed synchronisation of Sect. 1.3 (both conditions of Eq. 3), in GPU
 * form.  T sweeps are cut into passes of tile->t sweeps (t = 0: 1 sweep per
 * item); each item runs one pass on one block of k chunk q (tile->kchunk
 * planes, 0: 16).  Consecutive passes form segments of `team` passes
 * (1..1024), the GPU analog of a thread team: within a segment the items go
 * out in wavefronts, pass p on chunk q beside pass p+1 on chunk q - dl - 1,
 * so the passes of a segment stream through the grid a few chunks apart, as
 * the threads of a team follow each other through the blocks of a shared
 * cache; segments follow each other.  No cell is computed more often than
 * with tile->t sweeps per block (no halo is recomputed when t = 1).
 * Synchronisation (one counter per block; distances in k chunks, counted
 * beyond the one chunk of halo a pass needs from the pass before it; c_p =
 * chunks pass p has finished in a block column):
 *   c_{p-1} - c_p >= dl + 1  (lower bound: the data the item reads, plus
 *                            dl - 1 chunks of slack; dl >= 1),
 *   c_p - c_{p+1} <= du + 1  (upper bound, the pipeline's looseness; du = 0:
 *                            none, else du >= dl; dl = du = 1 is the paper's
 *                            lock-step case),
 * and a segment's front pass keeps dl + dt from the previous segment (dt,
 * the team delay, >= 0); the first pass has no lower and a segment's last
 * pass no upper condition.  sync == NULL: dl = 1, du = 0, dt = 0.  The
 * items also wait for the 27 neighbouring blocks of the previous pass.
 * The plan image has the layout of a one-grid batch: size it with
 * jacobi_pipelined_plan_bytes, copy it to the device, size the workspace
 * with jacobi_batched_workspace and run it with jacobi_batched_run in
 * JAC_BATCH_RELAXED mode (lockstep is refused, JAC_EARG).  a, b,
 * out_idx_host and the errors are as for jacobi_batched_plan with n = 1. */
typedef struct jac_pipeline {
    int32_t dl, du, dt;
} jac_pipeline_t;
size_t jacobi_pipelined_plan_bytes(int dtype, const jac_grid_t *g, int T,
                                   const jac_tile_t *tile);
int jacobi_pipelined_plan(int dtype, const jac_grid_t *g, void *a, void *b, int T,
                          int team, const jac_pipeline_t *sync,
                          const jac_tile_t *tile, void *plan_host,
                          size_t plan_bytes, int *out_idx_host);

/* Compressed single grid: T sweeps in ONE array instead of two, the
 * "compressed grid" of Sect. 1.3 (results written to a location shifted
 * against the one they were read from, alternate passes shifting back), with
 * t sweeps fused per pass as in jacobi_tblock.
 *  Layout: with S = tile->t (1..JAC_MAX_DEPTH, required: the layout depends
 *    on it) the array holds (nx+2+S) x (ny+2+S) x (nz+2) cells.  g gives the
 *    interior nx, ny, nz and the array's strides (0 = dense: sy = nx+2+S,
 *    sz = sy*(ny+2+S); else sy >= nx+2+S, sz >= sy*(ny+2+S)); u points at
 *    its element (0, 0, 0).  Frame 0 holds grid cell (i, j, k) at
 *    u[(i+S) + (j+S)*sy + k*sz], frame 1 at u[i + j*sy + k*sz].
 *  On entry frame 0 holds level 0 (shell included).  Pass p (ceil(T/t)
 *    passes, depths as for jacobi_tblock) reads frame p mod 2 and writes the
 *    other: the shift of (-S,-S,0) or (+S,+S,0) cells means that a block
 *    overwrites only inputs of its own and of its three neighbours on one
 *    side, so each workgroup waits, plane by plane, until those have read the
 *    plane it writes (per-block progress counters, bounded waits).  On
 *    return *out_frame = (number of passes) mod 2 names the frame holding
 *    level T, shell included, bitwise as jacobi_tblock computes it; the other
 *    elements of the array are undefined.  T = 0 enqueues nothing, frame 0.
 *  tile: t as above; bx, by, waves as for jacobi_tblock (64-wide blocks
 *    whose valid widths bx-2d and by-2d are at least d+t at every pass
 *    depth d, else JAC_EUNSUPPORTED; 0 = library choice); kchunk >= t or 0.
 *  ws: device workspace of jacobi_compressed_workspace(dtype, g, T, tile)
 *    bytes (0 on invalid arguments, see jacobi_last_error), 256-byte
 *    aligned, not overlapping the array: per-pass counters, copies of the
 *    2S+1 planes around each inner k chunk boundary, and the saved shell
 *    (about (2S+1)/kchunk of the array plus O(N^2)).  Its first int is an
 *    error flag: a wait that has not ended after about 2^20 polls gives up
 *    and sets it to 1 (results are then invalid); the caller may read it
 *    after synchronising. */
size_t jacobi_compressed_workspace(int dtype, const jac_grid_t *g, int T,
                                   const jac_tile_t *tile);
int jacobi_compressed(int dtype, const jac_grid_t *g, void *u, int T,
                      const jac_tile_t *tile, void *ws, size_t ws_bytes,
                      void *stream, int *out_frame);

/* Mixed-precision refinement helpers (outer FP64 loop around an FP32 Jacobi
 * inner solve; the refinement is not in the paper, the operator is the
 * Laplace system whose fixed point the Jacobi iteration of Sect. 1.1 seeks).
 * jacobi_residual_f64: r = (six neighbours of x, left to right) - 6*x in
 *   FP64 on the interior, i.e. b - A x for A = 6I - adjacency with the shell
 *   of x as Dirichlet data.  Writes (float)r into r32's interior (r32's shell
 *   is not written) and the squared 2-norm of the FP64 r into *norm2 (a
 *   device double), summed in a fixed order, so the result is identical run
 *   to run.  x and r32 share the geometry g (r32 holds floats).  ws: device
 *   workspace of at least jacobi_residual_workspace(g) bytes, 8-byte aligned.
 * jacobi_update_f64: x += (double)e32 on the interior.
 * jacobi_update_residual_f64: the update and the next residual in one pass
 *   over memory: x_new = x + (double)e32 on the interior (x_new's shell is
 *   not written: the caller keeps it equal to x's), then r32 and *norm2 as
 *   jacobi_residual_f64 computes them for x_new, and zero32's interior set to
 *   0 (zero32 is typically the next inner solve's starting guess).  x, e32,
 *   x_new, r32, zero32, norm2 and ws must not overlap (JAC_EARG); results
 *   are bitwise those of jacobi_update_f64 followed by jacobi_residual_f64
 *   (the norm's summation order differs).  ws as for jacobi_residual_f64.
 * jacobi_fill: every element of a grid, shell included, set to `value`
 *   (converted to the grid's dtype). */
size_t jacobi_residual_workspace(const jac_grid_t *g);
int jacobi_residual_f64(const jac_grid_t *g, const double *x, float *r32,
                        double *norm2, void *ws, size_t ws_bytes, void *stream);
int jacobi_update_residual_f64(const jac_grid_t *g, const double *x,
                               const float *e32, double *x_new, float *r32,
                               float *zero32, double *norm2, void *ws,
                               size_t ws_bytes, void *stream);
int jacobi_update_f64(const jac_grid_t *g, double *x, const float *e32,
                      void *stream);

/* jacobi_residual_f64 without a workspace, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments and results as jacobi_residual_f64
 * (bitwise: the same kernels), but the per-block partial sums of the norm go
 * to a fixed array of 2^17 doubles (1 MiB) that the library holds on each GPU
 * it runs on until the process ends.  The call allocates nothing and calls no
 * allocating routine.  Grids needing more partial sums,
 * ceil(nx/256) * ceil(ny/8) * ceil(nz/64) > 2^17 (e.g. beyond 2048^3), are
 * refused with JAC_EUNSUPPORTED before anything is enqueued.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or host threads) race and must be ordered by the
 * caller; consecutive calls on one stream are safe (each call writes every
 * partial sum it reads). */
int jacobi_residual_f64_noalloc(const jac_grid_t *g, const double *x, float *r32,
                                double *norm2, void *stream);
int jacobi_fill(int dtype, const jac_grid_t *g, void *x, double value,
                void *stream);

/* Device copy dst[0..bytes) = src[0..bytes), the STREAM-COPY-like kernel that
 * measures the bandwidth M_s of Eq. 2.  bytes must be a multiple of 16 and
 * both pointers 16-byte aligned; the ranges must not overlap. */
int jacobi_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Autotuner (the paper finds its blocking parameters experimentally,
 * Sect. 1.5): times jacobi_tblock for T sweeps on the caller's grids a and b
 * (whose contents it overwrites) for every menu block shape and depth
 * t = 1..tmax (0 = JAC_MAX_DEPTH) that fits the grid and compiles without
 * register spills, `reps` timed runs each after one warm-up, on `stream`
 * (synchronising it).  Writes the fastest choice to *best_host (kchunk = 0,
 * library choice) and its time per run in ms to *best_ms_host (may be NULL),
 * and remembers it (see the tuning cache below): later jacobi_tblock calls
 * on the same device architecture, dtype, geometry and T with t, bx, by all
 * 0 use it. */
int jacobi_autotune(int dtype, const jac_grid_t *g, void *a, void *b, int T,
                    int tmax, int reps, jac_tile_t *best_host,
                    float *best_ms_host, void *stream);

/* Tuning choices that outlive the process.  The library keeps the choices of
 * jacobi_autotune per (GPU architecture, dtype, nx, ny, nz, sy, sz, T); the
 * architecture is the device's name without feature flags ("gfx950").  A
 * choice for another architecture is kept but never used.  The cache file is
 * text, one choice a line, "arch dtype nx ny nz sy sz T t bx by waves kchunk
 * ms" (dtype f32 or f64; sy, sz as resolved, never 0; ms the measured time
 * per run), with '#' comment lines.  If the environment names a file in
 * JACOBI_TUNE_CACHE, the library reads it at its first lookup (a missing
 * file is no error; one that does not parse is reported on stderr and
 * ignored) and rewrites it after every successful jacobi_autotune.  Host
 * only; no HIP call except the one-time device query of the architecture.
 *  jacobi_tune_save: writes every remembered choice to path, replacing the
 *    file (through a temporary file in the same directory and a rename).
 *    JAC_EARG if it cannot be written.
 *  jacobi_tune_load: adds the choices in path (replacing remembered ones
 *    with the same key).  A line that does not parse, or names a dtype,
 *    depth or block shape the library does not have, is an error (JAC_EARG,
 *    the message names the line) and then nothing from the file is kept.
 *    *n_loaded (may be NULL) receives the number of choices read.
 *  jacobi_tune_lookup: the remembered choice for (arch, dtype, g, T) into
 *    *tile_host, or JAC_EUNSUPPORTED when there is none.  arch NULL: the
 *    current device's architecture.
 *  jacobi_tune_forget: forgets every remembered choice (the file, if any, is
 *    left alone). */
int jacobi_tune_save(const char *path);
int jacobi_tune_load(const char *path, int *n_loaded);
int jacobi_tune_lookup(const char *arch, int dtype, const jac_grid_t *g, int T,
                       jac_tile_t *tile_host);
int jacobi_tune_forget(void);

/* Supported block shapes for jacobi_tblock / jacobi_adjoint / batches: writes
 * up to `cap` triples (bx, by, waves) into shapes_host[3*n .. 3*n+2] and
 * returns the number available. */
int jacobi_tile_menu(int dtype, int *shapes_host, int cap);

/* The tile a call makes for (dtype, g, T, t) when tile fields are 0 (t = 0:
 * library choice of t as well).  kind 0: jacobi_tblock without a right-hand
 * side; 1: jacobi_tblock with one (those kernels hold one more value per cell
 * and level, so their register budget differs); 2: jacobi_adjoint (the trace
 * pass records the shell faces, a budget of its own).  Only nx, ny, nz of *g
 * are read.  Writes *tile_host; returns JAC_OK, or JAC_EARG for another kind. */
int jacobi_default_tile(int dtype, const jac_grid_t *g, int T, int t, int kind,
                        jac_tile_t *tile_host);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_H */
