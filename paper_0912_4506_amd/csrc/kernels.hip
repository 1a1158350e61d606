// Device kernels of libjacobi.so (gfx950 / CDNA4, wave64).
//
// The operation: sweeps of the 3D Jacobi update of Sect. 1.1 of the paper
// (average of the six face neighbours, fixed Dirichlet shell), and temporal
// blocking of t sweeps per pass over device memory.
//
// Arithmetic contract shared by every kernel: the six neighbours are summed
// left to right in the printed order (i-1, i+1, j-1, j+1, k-1, k+1); FP64
// divides by 6 with a correctly rounded quotient, FP32 multiplies by the
// float nearest 1/6.  The build uses -ffp-contract=off, so no add is fused.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "device_common.h"
#include "kernels.h"

namespace jac {

// ------------------------------------------------------------ plain sweep --
// One sweep, one pass over memory (the standard Jacobi of Sect. 1.1).  A block
// of NT threads (256 or 128) owns a strip of PLAIN_ROWS rows by 2*NT cells
// along i (two cells per thread) and streams through a chunk of k planes.  The strip's rows
// of plane k-1, k and k+1 stay in registers, so each step reads one new plane
// of the strip (PLAIN_ROWS + 2 whole row segments, contiguous in memory) and
// writes one; i-neighbours at the thread's ends are read through the cache.
// Coordinates of loads are clamped into the array; stores are predicated.
constexpr int PLAIN_ROWS = 8;

// Strip width: 512 cells (256 threads) unless 256-cell strips leave fewer
// idle lanes along i (e.g. nx = 256 or 768).
int plain_threads(int64_t nx)
{
    const int64_t idle512 = (nx + 511) / 512 * 512 - nx, idle256 = (nx + 255) / 256 * 256 - nx;
    return idle256 < idle512 ? 128 : 256;
}

template <typename real, int NT>
__global__ __launch_bounds__(NT) void plain_kernel(const real *__restrict__ A,
                                                   real *__restrict__ B, PlainArgs p)
{
    constexpr int RB = PLAIN_ROWS;
    // strips adjacent in j share their halo rows: keep them on one XCD's L2
    int bx, by, bz;
    remapped_block(bx, by, bz);
    const int i0 = 1 + bx * (2 * NT) + 2 * threadIdx.x;
    const int j0 = 1 + by * RB;
    const int k0 = 1 + bz * p.kchunk;
    const int k1 = min(k0 + p.kchunk, p.nz + 1);
    const int ia = min(i0, p.nx + 1), ib = min(i0 + 1, p.nx + 1);
    const int iw = min(i0 - 1, p.nx + 1), ie = min(i0 + 2, p.nx + 1);
    int64_t ro[RB + 2];
#pragma unroll
    for (int r = 0; r < RB + 2; ++r)
        ro[r] = (int64_t)min(j0 - 1 + r, p.ny + 1) * p.sy;

    // plane values of the strip: c = rows j0-1 .. j0+RB, two cells each;
    // w, e = the i-neighbours of the two cells, rows j0 .. j0+RB-1
    auto load = [&](int k, real(&c)[RB + 2][2], real(&w)[RB], real(&e)[RB]) {
        const real *pl = A + (int64_t)min(k, p.nz + 1) * p.sz;
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            c[r][0] = pl[ro[r] + ia];
            c[r][1] = pl[ro[r] + ib];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            w[r] = pl[ro[r + 1] + iw];
            e[r] = pl[ro[r + 1] + ie];
        }
    };
    real prev[RB][2], cur[RB + 2][2], cw[RB], ce[RB], nxt[RB + 2][2], nw[RB], ne[RB];
    load(k0 - 1, nxt, nw, ne);
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        prev[r][0] = nxt[r + 1][0];
        prev[r][1] = nxt[r + 1][1];
    }
    load(k0, cur, cw, ce);
    for (int k = k0; k < k1; ++k) {
        load(k + 1, nxt, nw, ne);
        // the same 2 x RB stores every step (cells outside the grid get the
        // drop offset), so the wait for the next plane skips the stores
        const auto rs = plane_rsrc(B + (int64_t)k * p.sz, (int)(p.sz * (int64_t)sizeof(real)));
        real sum[RB][2], q[RB][2];
        bool odd = false;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            real s0 = cw[r] + cur[r + 1][1];
            s0 = s0 + cur[r][0];
            s0 = s0 + cur[r + 2][0];
            s0 = s0 + prev[r][0];
            s0 = s0 + nxt[r + 1][0];
            real s1 = cur[r + 1][0] + ce[r];
            s1 = s1 + cur[r][1];
            s1 = s1 + cur[r + 2][1];
            s1 = s1 + prev[r][1];
            s1 = s1 + nxt[r + 1][1];
            sum[r][0] = s0;
            sum[r][1] = s1;
            q[r][0] = div6(s0);
            q[r][1] = div6(s1);
            odd = odd || div6_suspect(q[r][0]) || div6_suspect(q[r][1]);
        }
        // quotients the three-operation division may get wrong (NaN, Inf,
        // subnormal) are redone with IEEE division: one wave-uniform test per
        // step, so the plain sweep is IEEE-exact for every input
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(odd) != 0, 0)) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (div6_suspect(q[r][c]))
                        q[r][c] = div6_ieee(sum[r][c]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool row = j0 + r <= p.ny;
            const int o0 = row && i0 <= p.nx ? (int)((ro[r + 1] + i0) * (int64_t)sizeof(real))
                                             : kDropOffset;
            const int o1 = row && i0 + 1 <= p.nx
                               ? (int)((ro[r + 1] + i0 + 1) * (int64_t)sizeof(real))
                               : kDropOffset;
            plane_store(q[r][0], rs, o0);
            plane_store(q[r][1], rs, o1);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            prev[r][0] = cur[r + 1][0];
            prev[r][1] = cur[r + 1][1];
            cw[r] = nw[r];
            ce[r] = ne[r];
        }
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            cur[r][0] = nxt[r][0];
            cur[r][1] = nxt[r][1];
        }
    }
}

// ------------------------------------------------------------ small kernels --
// Copy the whole shell (faces, edges, corners) of grid a into grid b.
template <typename real>
__global__ void copy_shell_kernel(const real *__restrict__ a, real *__restrict__ b, GridArgs g)
{
    // one thread per (i, j) of the two k-faces, (i, k) of the j-faces and
    // (j, k) of the i-faces, over the full (n+2) extents
    const int64_t nxp = g.nx + 2, nyp = g.ny + 2, nzp = g.nz + 2;
    const int64_t nk = nxp * nyp, nj = nxp * nzp, ni = nyp * nzp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nk + nj + ni;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t o0, o1;
        if (t < nk) {
            const int64_t i = t % nxp, j = t / nxp;
            o0 = i + j * g.sy;
            o1 = o0 + (g.nz + 1) * g.sz;
        } else if (t < nk + nj) {
            const int64_t u = t - nk, i = u % nxp, k = u / nxp;
            o0 = i + k * g.sz;
            o1 = o0 + (g.ny + 1) * g.sy;
        } else {
            const int64_t u = t - nk - nj, j = u % nyp, k = u / nyp;
            o0 = j * g.sy + k * g.sz;
            o1 = o0 + (g.nx + 1);
        }
        b[o0] = a[o0];
        b[o1] = a[o1];
    }
}

// ------------------------------------------------- refinement (FP64 outer) --
// Residual of the Laplace system whose fixed point the Jacobi iteration seeks:
// r = (six neighbours of x, summed left to right) - 6x on the interior, FP64,
// i.e. b - A x for A = 6I - adjacency with the shell of x as Dirichlet data.
// Writes (float)r to r32 (interior) and a per-block partial sum of r^2.
// A block owns RB rows of 256 consecutive cells (one per thread) and streams
// a k chunk with the strip's k-1, k, k+1 rows in registers; each thread sums
// its cells' r^2 in stream order, the block sums its threads with a fixed
// tree, so the result is the same run to run.
//
// FUSED: the refinement's update comes first.  The grid the residual is taken
// of is xn = x + (double)e on the interior and x on the shell, formed on the
// fly at every stencil point; the kernel writes xn to xnew, the residual of
// xn, and zeroes the interior of z (the next inner solve's starting guess).
// x, e, xnew and z are distinct buffers, so no thread reads what another
// writes.
template <int RB, bool FUSED>
__global__ __launch_bounds__(256) void residual_kernel(const double *__restrict__ X,
                                                       const float *__restrict__ E,
                                                       double *__restrict__ xnew,
                                                       float *__restrict__ z,
                                                       float *__restrict__ r32,
                                                       double *__restrict__ partial, PlainArgs p)
{
    __shared__ double red[256];
    // one cell per thread: 256 consecutive cells of RB rows, streamed in k;
    // strips adjacent in j (sharing halo rows) stay on one XCD
    int bx, by, bz;
    remapped_block(bx, by, bz);
    const int i = 1 + bx * 256 + threadIdx.x;
    const int j0 = 1 + by * RB;
    const int k0 = 1 + bz * p.kchunk;
    const int k1 = min(k0 + p.kchunk, p.nz + 1);
    const int ic = min(i, p.nx + 1), iw = min(i - 1, p.nx + 1), ie = min(i + 1, p.nx + 1);
    // interior masks of the three i positions (FUSED only)
    const bool mc = ic <= p.nx, mw = iw >= 1 && iw <= p.nx, me = ie <= p.nx;
    int64_t ro[RB + 2];
    bool mj[RB + 2];
#pragma unroll
    for (int r = 0; r < RB + 2; ++r) {
        const int j = j0 - 1 + r;
        ro[r] = (int64_t)min(j, p.ny + 1) * p.sy;
        mj[r] = j >= 1 && j <= p.ny;
    }
    // both loads are unconditional (o is always inside the arrays), so they
    // issue back to back; the mask only selects
    auto value = [&](const double *xp, const float *ep, int64_t o, bool in) -> double {
        const double v = xp[o];
        if constexpr (FUSED) {
            const double u = v + (double)ep[o];
            return in ? u : v;
        } else {
            return v;
        }
    };
    // c: the RB+2 rows at i; w, e: the RB inner rows at i-1 and i+1
    auto load = [&](int k, double(&c)[RB + 2], double(&w)[RB], double(&e)[RB]) {
        const int kc = min(k, p.nz + 1);
        const double *pl = X + (int64_t)kc * p.sz;
        const float *el = E + (FUSED ? (int64_t)kc * p.sz : 0);
        const bool mk = kc >= 1 && kc <= p.nz;
#pragma unroll
        for (int r = 0; r < RB + 2; ++r)
            c[r] = value(pl, el, ro[r] + ic, mk && mj[r] && mc);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool m = mk && mj[r + 1];
            w[r] = value(pl, el, ro[r + 1] + iw, m && mw);
            e[r] = value(pl, el, ro[r + 1] + ie, m && me);
        }
    };
    double prev[RB], cur[RB + 2], cw[RB], ce[RB], nxt[RB + 2], nw[RB], ne[RB];
    load(k0 - 1, nxt, nw, ne);
#pragma unroll
    for (int r = 0; r < RB; ++r)
        prev[r] = nxt[r + 1];
    load(k0, cur, cw, ce);
    double acc = 0.0;
    for (int k = k0; k < k1; ++k) {
        load(k + 1, nxt, nw, ne);
        const int64_t po = (int64_t)k * p.sz;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            double s = cw[r] + ce[r];
            s = s + cur[r];
            s = s + cur[r + 2];
            s = s + prev[r];
            s = s + nxt[r + 1];
            const double six = 6.0 * cur[r + 1];
            const double v = s - six;
            if (j0 + r <= p.ny && i <= p.nx) {
                const int64_t o = po + ro[r + 1] + i;
                r32[o] = (float)v;
                acc = acc + v * v;
                if constexpr (FUSED) {
                    xnew[o] = cur[r + 1];
                    z[o] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            prev[r] = cur[r + 1];
            cw[r] = nw[r];
            ce[r] = ne[r];
        }
#pragma unroll
        for (int r = 0; r < RB + 2; ++r)
            cur[r] = nxt[r];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[((int64_t)bz * gridDim.y + by) * gridDim.x + bx] = red[0];
}

// Fill and update kernels: blocks own RES_ROWS rows x 256 cells and a k chunk
// of RES_KC planes, one cell per thread per row
constexpr int RES_ROWS = 4;
constexpr int RES_KC = 16;

// norm2 = sum of the n partials: each thread sums a strided subset in order,
// then a fixed tree over the 256 threads
__global__ __launch_bounds__(256) void sum_partials_kernel(const double *__restrict__ partial,
                                                           int64_t n, double *__restrict__ norm2)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += 256)
        acc = acc + partial[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *norm2 = red[0];
}

// every element (i, j, k) of a grid, shell included, set to v
template <typename real>
__global__ __launch_bounds__(256) void grid_fill_kernel(real *__restrict__ x, real v, GridArgs g)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * RES_ROWS;
    const int64_t k0 = (int64_t)blockIdx.z * RES_KC;
    if (i > g.nx + 1)
        return;
    for (int64_t k = k0; k < k0 + RES_KC && k <= g.nz + 1; ++k)
        for (int64_t j = j0; j < j0 + RES_ROWS && j <= g.ny + 1; ++j)
            x[i + j * g.sy + k * g.sz] = v;
}

// x += (double)e32 on the interior
__global__ __launch_bounds__(256) void update_kernel(double *__restrict__ x,
                                                     const float *__restrict__ e32, GridArgs g)
{
    const int64_t i = 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = 1 + (int64_t)blockIdx.y * RES_ROWS;
    const int64_t k0 = 1 + (int64_t)blockIdx.z * RES_KC;
    if (i > g.nx)
        return;
    for (int64_t k = k0; k < k0 + RES_KC && k <= g.nz; ++k)
        for (int64_t j = j0; j < j0 + RES_ROWS && j <= g.ny; ++j) {
            const int64_t o = i + j * g.sy + k * g.sz;
            x[o] = x[o] + (double)e32[o];
        }
}

// ------------------------------------------------------ shell face arrays --
// The six face layers of the shell as one compact array of F values:
// [i = 0 face: (k, j)], [i = nx+1 face], [j = 0 face: (k, i)], [j = ny+1 face],
// [k = 0 face: (j, i)], [k = nz+1 face], interior coordinates running fastest
// in the last index.  face_offset maps a face index to its grid element.
__device__ __forceinline__ int64_t face_offset(int64_t f, const GridArgs &g)
{
    const int64_t nyz = g.ny * g.nz, nxz = g.nx * g.nz;
    int64_t i, j, k;
    if (f < 2 * nyz) {
        const int64_t u = f % nyz;
        k = u / g.ny + 1;
        j = u % g.ny + 1;
        i = f < nyz ? 0 : g.nx + 1;
    } else if (f < 2 * nyz + 2 * nxz) {
        const int64_t v = f - 2 * nyz, u = v % nxz;
        k = u / g.nx + 1;
        i = u % g.nx + 1;
        j = v < nxz ? 0 : g.ny + 1;
    } else {
        const int64_t nxy = g.nx * g.ny, v = f - 2 * nyz - 2 * nxz, u = v % nxy;
        j = u / g.nx + 1;
        i = u % g.nx + 1;
        k = v < nxy ? 0 : g.nz + 1;
    }
    return i + j * g.sy + k * g.sz;
}

// faces[f] = grid[face f]
template <typename real>
__global__ void save_faces_kernel(const real *__restrict__ grid, real *__restrict__ faces,
                                  GridArgs g, int64_t F)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F;
         f += (int64_t)gridDim.x * blockDim.x)
        faces[f] = grid[face_offset(f, g)];
}

// grid[face f] = 0 (edges and corners of the shell untouched)
template <typename real>
__global__ void zero_faces_kernel(real *__restrict__ grid, GridArgs g, int64_t F)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F;
         f += (int64_t)gridDim.x * blockDim.x)
        grid[face_offset(f, g)] = real(0);
}

template <typename real>
__global__ void fill_kernel(real *__restrict__ x, int64_t n, real v)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
         f += (int64_t)gridDim.x * blockDim.x)
        x[f] = v;
}

// S[f] = (((S[f] + tr[0][f]) + tr[1][f]) + ...) over `depth` levels, in order
template <typename real>
__global__ void face_accum_kernel(real *__restrict__ S, const real *__restrict__ tr, int64_t F,
                                  int depth)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F;
         f += (int64_t)gridDim.x * blockDim.x) {
        real acc = S[f];
        for (int s = 0; s < depth; ++s)
            acc = acc + tr[(int64_t)s * F + f];
        S[f] = acc;
    }
}

// grid[face f] = G[f] + S[f] / 6
template <typename real>
__global__ void face_finalize_kernel(real *__restrict__ grid, const real *__restrict__ G,
                                     const real *__restrict__ S, GridArgs g, int64_t F)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < F;
         f += (int64_t)gridDim.x * blockDim.x)
        grid[face_offset(f, g)] = G[f] + div6_exact(S[f]);
}

// The whole shell of a grid (six faces with their edges and corners) as one
// compact array of shell_count(g) values: [k = 0 plane: (j, i)], [k = nz+1],
// [j = 0: (k, i)], [j = ny+1], [i = 0: (k, j)], [i = nx+1], each face over
// the full extents (edges and corners appear in several faces).
__device__ __forceinline__ int64_t shell_offset(int64_t f, const GridArgs &g)
{
    const int64_t nxp = g.nx + 2, nyp = g.ny + 2, nzp = g.nz + 2;
    const int64_t nk = nxp * nyp, nj = nxp * nzp, ni = nyp * nzp;
    if (f < 2 * nk) {
        const int64_t u = f % nk;
        return u % nxp + (u / nxp) * g.sy + (f < nk ? 0 : (g.nz + 1) * g.sz);
    }
    f -= 2 * nk;
    if (f < 2 * nj) {
        const int64_t u = f % nj;
        return u % nxp + (u / nxp) * g.sz + (f < nj ? 0 : (g.ny + 1) * g.sy);
    }
    f -= 2 * nj;
    const int64_t u = f % ni;
    return (u % nyp) * g.sy + (u / nyp) * g.sz + (f < ni ? 0 : g.nx + 1);
}

int64_t shell_count(const GridArgs &g)
{
    const int64_t nxp = g.nx + 2, nyp = g.ny + 2, nzp = g.nz + 2;
    return 2 * (nxp * nyp + nxp * nzp + nyp * nzp);
}

// save: store[f] = grid[shell f]; else grid[shell f] = store[f]
template <typename real>
__global__ __launch_bounds__(256) void shell_store_kernel(real *__restrict__ grid,
                                                          real *__restrict__ store, GridArgs g,
                                                          int64_t n, int save)
{
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = shell_offset(f, g);
        if (save)
            store[f] = grid[o];
        else
            grid[o] = store[f];
    }
}

// Shell copy a -> b of every grid of a batch: blockIdx.y is the grid.
template <typename real>
__global__ void batch_shell_kernel(const BatchGrid *__restrict__ grids)
{
    const BatchGrid G = grids[blockIdx.y];
    const GridArgs g{G.nx, G.ny, G.nz, G.sy, G.sz};
    const real *a = (const real *)G.a;
    real *b = (real *)G.b;
    const int64_t nxp = g.nx + 2, nyp = g.ny + 2, nzp = g.nz + 2;
    const int64_t nk = nxp * nyp, nj = nxp * nzp, ni = nyp * nzp;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nk + nj + ni;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t o0, o1;
        if (t < nk) {
            const int64_t i = t % nxp, j = t / nxp;
            o0 = i + j * g.sy;
            o1 = o0 + (g.nz + 1) * g.sz;
        } else if (t < nk + nj) {
            const int64_t u = t - nk, i = u % nxp, k = u / nxp;
            o0 = i + k * g.sz;
            o1 = o0 + (g.ny + 1) * g.sy;
        } else {
            const int64_t u = t - nk - nj, j = u % nyp, k = u / nyp;
            o0 = j * g.sy + k * g.sz;
            o1 = o0 + (g.nx + 1);
        }
        b[o0] = a[o0];
        b[o1] = a[o1];
    }
}

__global__ void zero_ints_kernel(int *__restrict__ x, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        x[t] = 0;
}

// dst = src for n 16-byte words: one word per thread, consecutive threads on
// consecutive words (the fastest copy form measured on MI355X)
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n)
        dst[t] = src[t];
}

// ------------------------------------------------------------------ launchers --
template <typename real>
hipError_t launch_plain(const real *a, real *b, const PlainArgs &p, hipStream_t st)
{
    const int nt = plain_threads(p.nx);
    dim3 grid((p.nx + 2 * nt - 1) / (2 * nt), (p.ny + PLAIN_ROWS - 1) / PLAIN_ROWS,
              (p.nz + p.kchunk - 1) / p.kchunk);
    if (nt == 256)
        hipLaunchKernelGGL((plain_kernel<real, 256>), grid, dim3(256), 0, st, a, b, p);
    else
        hipLaunchKernelGGL((plain_kernel<real, 128>), grid, dim3(128), 0, st, a, b, p);
    return hipGetLastError();
}

template <typename real>
static KernInfo tb_info(int cfg, int depth, int mode)
{
    constexpr bool f64 = sizeof(real) == 8;
    switch (mode) {
    case MODE_PLAIN: return f64 ? tb_info_plain_f64(cfg, depth) : tb_info_plain_f32(cfg, depth);
    case MODE_RHS: return f64 ? tb_info_rhs_f64(cfg, depth) : tb_info_rhs_f32(cfg, depth);
    case MODE_TRACE: return f64 ? tb_info_trace_f64(cfg, depth) : tb_info_trace_f32(cfg, depth);
    case MODE_COMP: return f64 ? tb_info_comp_f64(cfg, depth) : tb_info_comp_f32(cfg, depth);
    default: return KernInfo{nullptr, 0, 0};
    }
}

template <typename real>
hipError_t launch_tblock(int cfg, int depth, int mode, const TbArgs<real> &p, int nblocks,
                         hipStream_t st)
{
    const KernInfo ki = tb_info<real>(cfg, depth, mode);
    if (!ki.fn)
        return hipErrorInvalidValue;
    if (ki.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(ki.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ki.lds);
        if (e != hipSuccess)
            return e;
    }
    TbArgs<real> arg = p;
    void *args[] = {&arg};
    hipError_t e = hipLaunchKernel(ki.fn, dim3(nblocks), dim3(ki.threads), args, ki.lds, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the caller's next HIP call
        return e;
    }
    return hipGetLastError();
}

hipError_t launch_batched(int dtype, int cfg, int depth, int fixed, const BatchLaunch &L, int nblocks,
                          hipStream_t st)
{
    const KernInfo ki = dtype == 1 ? batch_info_f64(cfg, depth, fixed) : batch_info_f32(cfg, depth, fixed);
    if (!ki.fn)
        return hipErrorInvalidValue;
    if (ki.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(ki.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ki.lds);
        if (e != hipSuccess)
            return e;
    }
    BatchLaunch arg = L;
    void *args[] = {&arg};
    hipError_t e = hipLaunchKernel(ki.fn, dim3(nblocks), dim3(ki.threads), args, ki.lds, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the caller's next HIP call
        return e;
    }
    return hipGetLastError();
}

int batched_scratch(int dtype, int cfg, int depth, int fixed)
{
    const KernInfo ki = dtype == 1 ? batch_info_f64(cfg, depth, fixed) : batch_info_f32(cfg, depth, fixed);
    if (!ki.fn)
        return -1;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, ki.fn) != hipSuccess)
        return -1;
    return (int)attr.localSizeBytes;
}

int batched_occupancy(int dtype, int cfg, int depth, int fixed)
{
    const KernInfo ki = dtype == 1 ? batch_info_f64(cfg, depth, fixed) : batch_info_f32(cfg, depth, fixed);
    if (!ki.fn)
        return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ki.fn, ki.threads, ki.lds) != hipSuccess)
        return 0;
    return n;
}

int tblock_scratch(int dtype, int cfg, int depth, int mode)
{
    const KernInfo ki = dtype == 1 ? tb_info<double>(cfg, depth, mode)
                                   : tb_info<float>(cfg, depth, mode);
    if (!ki.fn)
        return -1;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, ki.fn) != hipSuccess)
        return -1;
    return (int)attr.localSizeBytes;
}

int tblock_occupancy(int dtype, int cfg, int depth, int mode)
{
    const KernInfo ki = dtype == 1 ? tb_info<double>(cfg, depth, mode)
                                   : tb_info<float>(cfg, depth, mode);
    if (!ki.fn)
        return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ki.fn, ki.threads, ki.lds) != hipSuccess)
        return 0;
    return n;
}

template <typename real>
hipError_t launch_copy_shell(const real *a, real *b, const GridArgs &g, hipStream_t st)
{
    const int64_t n = (g.nx + 2) * (g.ny + 2) + (g.nx + 2) * (g.nz + 2) + (g.ny + 2) * (g.nz + 2);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_shell_kernel<real>, dim3(blocks), dim3(256), 0, st, a, b, g);
    return hipGetLastError();
}

static dim3 strip_grid(const GridArgs &g)
{
    return dim3((unsigned)((g.nx + 255) / 256), (unsigned)((g.ny + RES_ROWS - 1) / RES_ROWS),
                (unsigned)((g.nz + RES_KC - 1) / RES_KC));
}

// Residual geometry: RB-row strips of 256 cells (RES_RB rows for the
// residual alone, FUSED_RB for the fused form, which loads twice as much per
// row), k chunks of RES_KCHUNK.  The partial sums are sized for the larger
// of the two grids.
static constexpr int RES_KCHUNK = 64;
static constexpr int RES_RB = 8;
static constexpr int FUSED_RB = 4;
static dim3 residual_grid(const GridArgs &g, int rb)
{
    return dim3((unsigned)((g.nx + 255) / 256), (unsigned)((g.ny + rb - 1) / rb),
                (unsigned)((g.nz + RES_KCHUNK - 1) / RES_KCHUNK));
}

int64_t residual_partials(const GridArgs &g)
{
    const dim3 d = residual_grid(g, FUSED_RB);  // the larger of the two grids
    return (int64_t)d.x * d.y * d.z;
}

// ------------------------------------------------ allocation-free residual --
// Device memory of jacobi_residual_f64_noalloc: the per-block partial sums of
// the residual norm, in a fixed array instead of a caller's workspace.  Each
// GPU the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, not the device array: the device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is passed to kernels.
constexpr int64_t kNoAllocPartials = int64_t(1) << 17;  // 1 MiB of doubles
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device
}  // namespace

int64_t noalloc_partials_max() { return kNoAllocPartials; }

int64_t residual_partials_plain(const GridArgs &g)
{
    const dim3 d = residual_grid(g, RES_RB);
    return (int64_t)d.x * d.y * d.z;
}

hipError_t noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;  // looked up with device `dev` current
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

static hipError_t sum_partials(const double *partial, const dim3 &grid, double *norm2,
                               hipStream_t st)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, partial,
                       (int64_t)grid.x * grid.y * grid.z, norm2);
    return hipGetLastError();
}

hipError_t launch_residual(const double *x, float *r32, double *partial, double *norm2,
                           const GridArgs &g, hipStream_t st)
{
    const dim3 grid = residual_grid(g, RES_RB);
    PlainArgs p{(int)g.nx, (int)g.ny, (int)g.nz, RES_KCHUNK, g.sy, g.sz};
    hipLaunchKernelGGL((residual_kernel<RES_RB, false>), grid, dim3(256), 0, st, x, nullptr,
                       nullptr, nullptr, r32, partial, p);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_partials(partial, grid, norm2, st);
}

hipError_t launch_update_residual(const double *x, const float *e32, double *xnew, float *z,
                                  float *r32, double *partial, double *norm2, const GridArgs &g,
                                  hipStream_t st)
{
    const dim3 grid = residual_grid(g, FUSED_RB);
    PlainArgs p{(int)g.nx, (int)g.ny, (int)g.nz, RES_KCHUNK, g.sy, g.sz};
    hipLaunchKernelGGL((residual_kernel<FUSED_RB, true>), grid, dim3(256), 0, st, x, e32, xnew, z,
                       r32, partial, p);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_partials(partial, grid, norm2, st);
}

hipError_t launch_update(double *x, const float *e32, const GridArgs &g, hipStream_t st)
{
    hipLaunchKernelGGL(update_kernel, strip_grid(g), dim3(256), 0, st, x, e32, g);
    return hipGetLastError();
}

// a dense grid is one contiguous run of span elements: fill it flat
template <typename real>
__global__ __launch_bounds__(256) void flat_fill_kernel(real *__restrict__ x, int64_t n, real v)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    constexpr int PER = 16 / sizeof(real);
    const int64_t base = t * PER;
    if (base + PER <= n) {
        typedef real vec __attribute__((ext_vector_type(PER)));
        vec w;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            w[q] = v;
        *reinterpret_cast<vec *>(x + base) = w;
    } else {
        for (int64_t q = base; q < n; ++q)
            x[q] = v;
    }
}

template <typename real>
hipError_t launch_grid_fill(real *x, real v, const GridArgs &g, hipStream_t st)
{
    if (g.sy == g.nx + 2 && g.sz == g.sy * (g.ny + 2) && ((uintptr_t)x % 16) == 0) {
        const int64_t n = g.sz * (g.nz + 2);
        const int64_t per = 16 / (int64_t)sizeof(real);
        const int64_t blocks = ((n + per - 1) / per + 255) / 256;
        hipLaunchKernelGGL(flat_fill_kernel<real>, dim3((unsigned)blocks), dim3(256), 0, st, x, n, v);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((g.nx + 2 + 255) / 256), (unsigned)((g.ny + 2 + RES_ROWS - 1) / RES_ROWS),
                    (unsigned)((g.nz + 2 + RES_KC - 1) / RES_KC));
    hipLaunchKernelGGL(grid_fill_kernel<real>, grid, dim3(256), 0, st, x, v, g);
    return hipGetLastError();
}
template hipError_t launch_grid_fill<float>(float *, float, const GridArgs &, hipStream_t);
template hipError_t launch_grid_fill<double>(double *, double, const GridArgs &, hipStream_t);

// dst += src on every element (i, j, k) of a grid, shell included
template <typename real>
__global__ __launch_bounds__(256) void grid_add_kernel(real *__restrict__ dst,
                                                       const real *__restrict__ src, GridArgs g)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * RES_ROWS;
    const int64_t k0 = (int64_t)blockIdx.z * RES_KC;
    if (i > g.nx + 1)
        return;
    for (int64_t k = k0; k < k0 + RES_KC && k <= g.nz + 1; ++k)
        for (int64_t j = j0; j < j0 + RES_ROWS && j <= g.ny + 1; ++j) {
            const int64_t c = i + j * g.sy + k * g.sz;
            dst[c] = dst[c] + src[c];
        }
}

// the same on a dense grid, as one contiguous run of n elements, 16 bytes a thread
template <typename real>
__global__ __launch_bounds__(256) void flat_add_kernel(real *__restrict__ dst,
                                                       const real *__restrict__ src, int64_t n)
{
    constexpr int PER = 16 / sizeof(real);
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PER;
    if (base + PER <= n) {
        typedef real vec __attribute__((ext_vector_type(PER)));
        const vec a = *reinterpret_cast<const vec *>(dst + base);
        const vec b = *reinterpret_cast<const vec *>(src + base);
        vec w;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            w[q] = a[q] + b[q];
        *reinterpret_cast<vec *>(dst + base) = w;
    } else {
        for (int64_t q = base; q < n; ++q)
            dst[q] = dst[q] + src[q];
    }
}

template <typename real>
hipError_t launch_grid_add(real *dst, const real *src, const GridArgs &g, hipStream_t st)
{
    if (g.sy == g.nx + 2 && g.sz == g.sy * (g.ny + 2) && ((uintptr_t)dst % 16) == 0 &&
        ((uintptr_t)src % 16) == 0) {
        const int64_t n = g.sz * (g.nz + 2);
        const int64_t per = 16 / (int64_t)sizeof(real);
        const int64_t blocks = ((n + per - 1) / per + 255) / 256;
        hipLaunchKernelGGL(flat_add_kernel<real>, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((g.nx + 2 + 255) / 256), (unsigned)((g.ny + 2 + RES_ROWS - 1) / RES_ROWS),
                    (unsigned)((g.nz + 2 + RES_KC - 1) / RES_KC));
    hipLaunchKernelGGL(grid_add_kernel<real>, grid, dim3(256), 0, st, dst, src, g);
    return hipGetLastError();
}
template hipError_t launch_grid_add<float>(float *, const float *, const GridArgs &, hipStream_t);
template hipError_t launch_grid_add<double>(double *, const double *, const GridArgs &, hipStream_t);

static int grid_blocks(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

template <typename real>
hipError_t launch_faces(int op, real *grid, real *G, real *S, const real *tr, const GridArgs &g,
                        int64_t F, int depth, hipStream_t st)
{
    const int nb = grid_blocks(F);
    switch (op) {
    case FACES_SAVE:
        hipLaunchKernelGGL(save_faces_kernel<real>, dim3(nb), dim3(256), 0, st, grid, G, g, F);
        break;
    case FACES_ZERO:
        hipLaunchKernelGGL(zero_faces_kernel<real>, dim3(nb), dim3(256), 0, st, grid, g, F);
        break;
    case FACES_CLEAR_SUM:
        hipLaunchKernelGGL(fill_kernel<real>, dim3(nb), dim3(256), 0, st, S, F, real(0));
        break;
    case FACES_ACCUM:
        hipLaunchKernelGGL(face_accum_kernel<real>, dim3(nb), dim3(256), 0, st, S, tr, F, depth);
        break;
    case FACES_FINALIZE:
        hipLaunchKernelGGL(face_finalize_kernel<real>, dim3(nb), dim3(256), 0, st, grid, G, S, g, F);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename real>
hipError_t launch_batch_shells(const BatchGrid *grids, int n, int64_t max_shell, hipStream_t st)
{
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((max_shell + 255) / 256, 64));
    hipLaunchKernelGGL(batch_shell_kernel<real>, dim3(bx, n), dim3(256), 0, st, grids);
    return hipGetLastError();
}
template hipError_t launch_batch_shells<float>(const BatchGrid *, int, int64_t, hipStream_t);
template hipError_t launch_batch_shells<double>(const BatchGrid *, int, int64_t, hipStream_t);

template <typename real>
hipError_t launch_shell_store(int save, real *grid, real *store, const GridArgs &g, hipStream_t st)
{
    const int64_t n = shell_count(g);
    hipLaunchKernelGGL(shell_store_kernel<real>, dim3(grid_blocks(n)), dim3(256), 0, st, grid,
                       store, g, n, save);
    return hipGetLastError();
}
template hipError_t launch_shell_store<float>(int, float *, float *, const GridArgs &, hipStream_t);
template hipError_t launch_shell_store<double>(int, double *, double *, const GridArgs &,
                                               hipStream_t);

hipError_t launch_zero_ints(int *x, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_blocks(n)), dim3(256), 0, st, x, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4 *)src,
                       (uint4 *)dst, n);
    return hipGetLastError();
}

template hipError_t launch_plain<float>(const float *, float *, const PlainArgs &, hipStream_t);
template hipError_t launch_plain<double>(const double *, double *, const PlainArgs &, hipStream_t);
template hipError_t launch_tblock<float>(int, int, int, const TbArgs<float> &, int, hipStream_t);
template hipError_t launch_tblock<double>(int, int, int, const TbArgs<double> &, int, hipStream_t);
template hipError_t launch_faces<float>(int, float *, float *, float *, const float *,
                                       const GridArgs &, int64_t, int, hipStream_t);
template hipError_t launch_faces<double>(int, double *, double *, double *, const double *,
                                        const GridArgs &, int64_t, int, hipStream_t);
template hipError_t launch_copy_shell<float>(const float *, float *, const GridArgs &, hipStream_t);
template hipError_t launch_copy_shell<double>(const double *, double *, const GridArgs &, hipStream_t);

}  // namespace jac
