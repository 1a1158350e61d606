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

#include "kernels.h"

namespace jac {

// ---------------------------------------------------------------- division --
// Correctly rounded s/6 in three operations (Markstein's correction step):
// q0 = s * fl(1/6) is within one ulp of s/6, the residual s - 6 q0 is exact in
// an FMA, and q0 + r * fl(1/6) rounds to the correctly rounded quotient
// (P. Markstein, IBM J. Res. Dev. 34(1), 1990; Muller et al., Handbook of
// Floating-Point Arithmetic, division by a correctly rounded reciprocal).
// Valid away from overflow and underflow, i.e. for |s| in [2^-1020, 2^1020]
// and s = 0; the tests compare it bitwise with IEEE division.
__device__ __forceinline__ double div6(double s)
{
    const double c = 0x1.5555555555555p-3;  // the double nearest 1/6
    const double q = s * c;
    const double r = __fma_rn(-6.0, q, s);
    return __fma_rn(r, c, q);
}

__device__ __forceinline__ float div6(float s)
{
    return s * (1.0f / 6.0f);
}

// ------------------------------------------------------- cross-lane moves --
// DPP wave shifts (GFX9 wave_shr:1 / wave_shl:1): lane l receives the value
// of lane l-1 (shr) or l+1 (shl); bound_ctrl makes the lane with no source
// read 0, so no old value has to be materialised.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
    const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    return __hiloint2double(h2, l2);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <typename real>
__device__ __forceinline__ real from_left(real v) { return dpp_move<DPP_WAVE_SHR1>(v); }
template <typename real>
__device__ __forceinline__ real from_right(real v) { return dpp_move<DPP_WAVE_SHL1>(v); }

// ------------------------------------------------------------ plain sweep --
// One sweep, one pass over memory (the standard Jacobi of Sect. 1.1).  A block
// of 64 x 4 threads owns 64 x 4 interior columns and a chunk of k planes; each
// thread keeps its column's k-1, k, k+1 values in registers and reads the four
// in-plane neighbours through the cache.
template <typename real>
__global__ __launch_bounds__(256) void plain_kernel(const real *__restrict__ A,
                                                    real *__restrict__ B,
                                                    PlainArgs p)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63) + 1;
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6) + 1;
    const int k0 = blockIdx.z * p.kchunk + 1;
    const int k1 = min(k0 + p.kchunk, p.nz + 1);
    if (i > p.nx || j > p.ny)
        return;
    const int64_t col = (int64_t)i + (int64_t)j * p.sy;
    const real *a = A + col;
    real *b = B + col;
    real below = a[(int64_t)(k0 - 1) * p.sz];
    real centre = a[(int64_t)k0 * p.sz];
    for (int k = k0; k < k1; ++k) {
        const int64_t o = (int64_t)k * p.sz;
        const real above = a[o + p.sz];
        real s = a[o - 1];
        s = s + a[o + 1];
        s = s + a[o - p.sy];
        s = s + a[o + p.sy];
        s = s + below;
        s = s + above;
        b[o] = div6(s);
        below = centre;
        centre = above;
    }
}

// -------------------------------------------------- temporally blocked pass --
// Block placement along one axis.  Blocks are w cells wide including a halo
// of h cells per side.  Block 0 starts at the shell cell 0, which passes its
// value through unchanged at every level, so it needs no halo on that side:
// its valid range is [1, w - h).  Block b >= 1 is valid on [a, a + w - 2h)
// and starts at e = a - h.  Valid ranges tile [1, n] without overlap.
struct AxisTile {
    int e, a, b;  // first cell of the block; valid cells [a, b)
};

__device__ __forceinline__ AxisTile axis_tile(int blk, int n, int w, int h)
{
    const int first = w - h, mid = w - 2 * h;
    AxisTile t;
    if (blk == 0) {
        t.e = 0;
        t.a = 1;
        t.b = first;
    } else {
        t.a = first + (blk - 1) * mid;
        t.e = t.a - h;
        t.b = t.a + mid;
    }
    t.b = min(t.b, n + 1);
    return t;
}

// Workgroup ids reach the eight XCDs round robin (id mod 8), and each XCD has
// its own L2.  Remap so that XCD x works through a contiguous range of
// logical blocks: blocks that share halo cells then run on the same L2 at the
// same time.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, rem = n & 7, x = b & 7, idx = b >> 3;
    return x * q + min(x, rem) + idx;
}

// The exchange buffer is double-buffered (one barrier per stream step) when
// two copies fit in the 160 KiB of LDS a gfx950 workgroup may use.
template <typename real, int TL, int CI, int W>
constexpr bool xch_double()
{
    return 2 * (W * 2 * TL * CI * 64) * sizeof(real) <= 160 * 1024;
}

template <typename real, int TL, int CI, int W>
constexpr size_t xch_bytes()
{
    return (xch_double<real, TL, CI, W>() ? 2 : 1) * (size_t)(W * 2 * TL * CI * 64) * sizeof(real);
}

// One pass fuses TL sweeps.  A workgroup of W waves owns an extended block of
// (64*CI) x (W*R) cells in (i, j): lane l of wave w holds cells
// i = e_i + CI*l + c (c < CI) and j = e_j + w*R + r (r < R) in registers.  The
// block streams through k.  At stream step k, level 0 (the input) supplies
// plane k and level s (1..TL) completes plane k - s, so the levels form a
// wavefront skewed by one plane per level.  Halo cells are recomputed: the
// valid part of level s shrinks by one cell per side and level (the rule that
// update s covers a region h - s layers larger, Sect. 2.1), and the block
// writes only its valid cells.
//
// Per level s and cell the kernel keeps two values:
//   Q = level s-1 at the plane being completed (it is the k-1 term of the next
//       plane, and the value a shell cell passes through), and
//   P = ((((W + E) + S) + N) + D) of that plane, the first five terms of the
//       update in the printed order (D = the k-1 neighbour).
// When level s-1 delivers the next plane U, level s completes its plane as
// (P + U) / 6 -- the full left-to-right sum -- with no neighbour exchange, so
// the levels run back to back.  Then the newly delivered planes of all levels
// are exchanged at once (i-neighbours by DPP wave shifts, j-neighbours from
// registers, and across wave boundaries through LDS) and P, Q advance.  The
// stream loop is unrolled twice with the two Q sets swapping roles, so no
// register copies carry Q from one step to the next.
// Loads clamp their coordinates into the array: cells outside it hold
// garbage that only ever reaches other outside cells or shell cells, and
// shell cells (i, j or k = 0 or n+1) pass their value through at every level.
template <typename real, int TL, int CI, int R, int W, int MODE>
__global__ __launch_bounds__(64 * W) void tblock_kernel(TbArgs<real> p)
{
    static_assert(TL >= 1 && TL <= JAC_MAX_DEPTH_DEV, "depth");
    extern __shared__ unsigned char smem_raw[];
    real *xch = reinterpret_cast<real *>(smem_raw);  // [2][W][2][TL][CI][64]

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int bid = xcd_remap(blockIdx.x, p.nti * p.ntj * p.nkc);
    const int ti = bid % p.nti;
    const int tj = (bid / p.nti) % p.ntj;
    const int tk = bid / (p.nti * p.ntj);
    const AxisTile xi = axis_tile(ti, p.nx, 64 * CI, p.hi);
    const AxisTile xj = axis_tile(tj, p.ny, W * R, TL);
    const int k0 = 1 + tk * p.kchunk;
    const int k1 = min(k0 + p.kchunk, p.nz + 1);
    const int kstart = max(k0 - TL, 0);
    const int nsteps = ((k1 - 1 + TL) - kstart + 2) & ~1;  // rounded up to even

    // per-lane columns
    int ic[CI];
    bool sh_i[CI], ok_i[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) {
        const int i = xi.e + CI * lane + c;
        ic[c] = min(max(i, 0), p.nx + 1);
        sh_i[c] = i == 0 || i == p.nx + 1;
        ok_i[c] = i >= xi.a && i < xi.b;
    }
    const bool fix_i = xi.e <= 0 || xi.e + 64 * CI - 1 >= p.nx + 1;
    // per-wave rows (uniform)
    int64_t rowoff[R];
    bool sh_j[R], ok_j[R];
    bool fix_j = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = xj.e + w * R + r;
        rowoff[r] = (int64_t)min(max(j, 0), p.ny + 1) * p.sy;
        sh_j[r] = j == 0 || j == p.ny + 1;
        ok_j[r] = j >= xj.a && j < xj.b;
        fix_j = fix_j || sh_j[r];
    }

    auto load_plane = [&](const real *__restrict__ src, int k, real(&v)[R][CI]) {
        const real *plane = src + (int64_t)min(max(k, 0), p.nz + 1) * p.sz;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const real *row = plane + rowoff[r];
#pragma unroll
            for (int c = 0; c < CI; ++c)
                v[r][c] = row[ic[c]];
        }
    };

    real P[TL][R][CI], QA[TL][R][CI], QB[TL][R][CI];
#pragma unroll
    for (int s = 0; s < TL; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                P[s][r][c] = real(0);
                QA[s][r][c] = real(0);
                QB[s][r][c] = real(0);
            }
    constexpr int NRW = MODE == MODE_RHS ? TL : 1;
    real rw[NRW][R][CI];  // rw[s] = rhs at plane k-1-s (MODE_RHS)
    real rnext[R][CI];
#pragma unroll
    for (int s = 0; s < NRW; ++s)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < CI; ++c)
                rw[s][r][c] = real(0);
    if constexpr (MODE == MODE_RHS)
        load_plane(p.rhs, kstart - 1, rnext);

    real CA[R][CI], CB[R][CI];
    load_plane(p.src, kstart, CA);

    const int wa = w > 0 ? w - 1 : w;      // wave holding row j-1 of row 0
    const int wb = w < W - 1 ? w + 1 : w;  // wave holding row j+1 of row R-1
    // exchange buffer: one or two parities of [W][2 rows][TL][CI][64 lanes]
    constexpr int XSLAB = W * 2 * TL * CI * 64;
    constexpr bool DBUF = xch_double<real, TL, CI, W>();
    auto xidx = [](int wv, int side, int s, int c, int ln) {
        return (((wv * 2 + side) * TL + s) * CI + c) * 64 + ln;
    };
    for (int n = threadIdx.x; n < (DBUF ? 2 : 1) * XSLAB; n += 64 * W)
        xch[n] = real(0);
    __syncthreads();
    // i-neighbours of a row of CI cells: DPP across lanes at the ends
    auto neighbours_i = [](const real(&x)[CI], real(&west)[CI], real(&east)[CI]) {
        west[0] = from_left(x[CI - 1]);
        east[CI - 1] = from_right(x[0]);
#pragma unroll
        for (int c = 1; c < CI; ++c)
            west[c] = x[c - 1];
#pragma unroll
        for (int c = 0; c < CI - 1; ++c)
            east[c] = x[c + 1];
    };

    // One stream step: Qi = Q carried in, Qo = Q carried out (the planes
    // delivered this step), cur = plane k of level 0, nxt = prefetch of k+1.
    auto step = [&](int k, real(&Qi)[TL][R][CI], real(&Qo)[TL][R][CI], real(&cur)[R][CI],
                    real(&nxt)[R][CI]) {
        load_plane(p.src, k + 1, nxt);
        if constexpr (MODE == MODE_RHS) {
#pragma unroll
            for (int s = NRW - 1; s > 0; --s)
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < CI; ++c)
                        rw[s][r][c] = rw[s - 1][r][c];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < CI; ++c)
                    rw[0][r][c] = rnext[r][c];
            load_plane(p.rhs, k, rnext);
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < CI; ++c)
                Qo[0][r][c] = cur[r][c];

        // ---- complete one plane per level, back to back; right after level s
        // completes, advance P[s-1] for the rows whose j-neighbours are in
        // registers.  The wave's first and last rows are finished after the
        // exchange; their Q values live in LDS (own slot, previous parity).
        const int par = DBUF ? (k & 1) : 0;
        real *xcur = xch + par * XSLAB;
        const real *xold = xch + (DBUF ? (par ^ 1) : 0) * XSLAB;
#pragma unroll
        for (int s = 1; s <= TL; ++s) {
            const int plane = k - s;
            real o[R][CI];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    real sum = P[s - 1][r][c] + Qo[s - 1][r][c];
                    if constexpr (MODE == MODE_RHS)
                        sum = sum + rw[s - 1][r][c];
                    o[r][c] = div6(sum);
                }
            // pass-through value of a shell cell: its level s-1 value
            auto qin = [&](int r, int c) -> real {
                if (r == 0)
                    return xold[xidx(w, 0, s - 1, c, lane)];
                if (r == R - 1)
                    return xold[xidx(w, 1, s - 1, c, lane)];
                return Qi[s - 1][r][c];
            };
            if (fix_i) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < CI; ++c)
                        if (sh_i[c])
                            o[r][c] = qin(r, c);
            }
            const bool sh_plane = plane == 0 || plane == p.nz + 1;
            if (sh_plane || fix_j) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (sh_plane || sh_j[r]) {
#pragma unroll
                        for (int c = 0; c < CI; ++c)
                            o[r][c] = qin(r, c);
                    }
            }
            if (s < TL) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < CI; ++c)
                        Qo[s][r][c] = o[r][c];
            } else if (plane >= k0 && plane < k1) {
                real *dplane = p.dst + (int64_t)plane * p.sz;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (ok_j[r]) {
                        real *row = dplane + rowoff[r];
#pragma unroll
                        for (int c = 0; c < CI; ++c)
                            if (ok_i[c])
                                row[ic[c]] = o[r][c];
                    }
            }
            // advance P[s-1] (rows 1 .. R-2) from the plane delivered to level s
            const int l = s - 1;
#pragma unroll
            for (int r = 1; r < R - 1; ++r) {
                real west[CI], east[CI];
                neighbours_i(Qo[l][r], west, east);
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    real q = west[c] + east[c];
                    q = q + Qo[l][r - 1][c];
                    q = q + Qo[l][r + 1][c];
                    P[l][r][c] = q + Qi[l][r][c];
                }
            }
        }

        // ---- publish the wave's first and last rows, then finish their P.
        // With one buffer, the old rows are read back before they are
        // overwritten, and a barrier keeps the previous step's readers safe.
        real dold[TL][2][CI];
        if constexpr (!DBUF) {
#pragma unroll
            for (int s = 0; s < TL; ++s)
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    dold[s][0][c] = xold[xidx(w, 0, s, c, lane)];
                    dold[s][1][c] = xold[xidx(w, 1, s, c, lane)];
                }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < TL; ++s)
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                xcur[xidx(w, 0, s, c, lane)] = Qo[s][0][c];
                xcur[xidx(w, 1, s, c, lane)] = Qo[s][R - 1][c];
            }
        __syncthreads();
        auto dprev = [&](int side, int s, int c) -> real {
            if constexpr (DBUF)
                return xold[xidx(w, side, s, c, lane)];
            else
                return dold[s][side][c];
        };
#pragma unroll
        for (int s = 0; s < TL; ++s) {
            real west[CI], east[CI];
            neighbours_i(Qo[s][0], west, east);
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                const real sn = xcur[xidx(wa, 1, s, c, lane)];
                const real north = R > 1 ? Qo[s][R > 1 ? 1 : 0][c] : xcur[xidx(wb, 0, s, c, lane)];
                real q = west[c] + east[c];
                q = q + sn;
                q = q + north;
                P[s][0][c] = q + dprev(0, s, c);
            }
            if constexpr (R > 1) {
                neighbours_i(Qo[s][R - 1], west, east);
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    const real nn = xcur[xidx(wb, 0, s, c, lane)];
                    real q = west[c] + east[c];
                    q = q + Qo[s][R - 2][c];
                    q = q + nn;
                    P[s][R - 1][c] = q + dprev(1, s, c);
                }
            }
        }
    };

    for (int n = 0; n < nsteps; n += 2) {
        step(kstart + n, QA, QB, CA, CB);
        step(kstart + n + 1, QB, QA, CB, CA);
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

// dst = src for bytes/16 16-byte words (grid-stride, coalesced)
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride)
        dst[t] = src[t];
}

// ------------------------------------------------------------------ launchers --
template <typename real>
hipError_t launch_plain(const real *a, real *b, const PlainArgs &p, hipStream_t st)
{
    dim3 grid((p.nx + 63) / 64, (p.ny + 3) / 4, (p.nz + p.kchunk - 1) / p.kchunk);
    hipLaunchKernelGGL(plain_kernel<real>, grid, dim3(256), 0, st, a, b, p);
    return hipGetLastError();
}

struct KernInfo {
    const void *fn;
    size_t lds;
    int threads;
};

template <typename real, int TL, int CI, int R, int W, int MODE>
static KernInfo tb_info_one()
{
    return KernInfo{(const void *)tblock_kernel<real, TL, CI, R, W, MODE>,
                    xch_bytes<real, TL, CI, W>(), 64 * W};
}

template <typename real, int CI, int R, int W, int MODE>
static KernInfo tb_info_depth(int depth)
{
    switch (depth) {
    case 1: return tb_info_one<real, 1, CI, R, W, MODE>();
    case 2: return tb_info_one<real, 2, CI, R, W, MODE>();
    case 3: return tb_info_one<real, 3, CI, R, W, MODE>();
    case 4: return tb_info_one<real, 4, CI, R, W, MODE>();
    case 5: return tb_info_one<real, 5, CI, R, W, MODE>();
    case 6: return tb_info_one<real, 6, CI, R, W, MODE>();
    case 7: return tb_info_one<real, 7, CI, R, W, MODE>();
    case 8: return tb_info_one<real, 8, CI, R, W, MODE>();
    default: return KernInfo{nullptr, 0, 0};
    }
}

template <typename real>
static KernInfo tb_info(int cfg, int depth, int mode)
{
#define JAC_CFG(ID, CI, R, W)                                                  \
    case ID:                                                                   \
        return mode == MODE_RHS ? tb_info_depth<real, CI, R, W, MODE_RHS>(depth) \
                                : tb_info_depth<real, CI, R, W, MODE_PLAIN>(depth);
    switch (cfg) {
        JAC_TILE_MENU(JAC_CFG)
    default: return KernInfo{nullptr, 0, 0};
    }
#undef JAC_CFG
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
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
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

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 256 * 16);
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, st, (const uint4 *)src,
                       (uint4 *)dst, n);
    return hipGetLastError();
}

template hipError_t launch_plain<float>(const float *, float *, const PlainArgs &, hipStream_t);
template hipError_t launch_plain<double>(const double *, double *, const PlainArgs &, hipStream_t);
template hipError_t launch_tblock<float>(int, int, int, const TbArgs<float> &, int, hipStream_t);
template hipError_t launch_tblock<double>(int, int, int, const TbArgs<double> &, int, hipStream_t);
template hipError_t launch_copy_shell<float>(const float *, float *, const GridArgs &, hipStream_t);
template hipError_t launch_copy_shell<double>(const double *, double *, const GridArgs &, hipStream_t);

}  // namespace jac
