// The temporally blocked pass (a template instantiated per dtype and mode in
// tb_*.hip).  Arithmetic contract: the six neighbours are summed left to
// right in the printed order (i-1, i+1, j-1, j+1, k-1, k+1); FP64 divides by 6
// with a correctly rounded quotient, FP32 multiplies by the float nearest 1/6.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace jac {

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

// The exchange buffer is double-buffered (one barrier per stream step) when
// two copies fit in the 160 KiB of LDS a gfx950 workgroup may use, less 1 KiB
// kept for the kernels' static LDS.
template <typename real, int TL, int CI, int W>
constexpr bool xch_double()
{
    return 2 * (W * 2 * TL * CI * 64) * sizeof(real) <= 159 * 1024;
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
// registers, and across wave boundaries through LDS) and P, Q advance.
// Q is carried from one step to the next by copying the new set back after
// every step: one move per value.  (Unrolling the loop twice with the two
// sets swapping roles needs no copies, but the compiler then keeps about 50
// more VGPRs live, and the register budget is what limits the block.)
// Loads clamp their coordinates into the array: cells outside it hold
// garbage that only ever reaches other outside cells or shell cells, and
// shell cells (i, j or k = 0 or n+1) pass their value through at every level.
// Output planes [k0, k1) of block column (ti, tj) for one pass at `depth`
// <= TL levels (the block geometry is planned for TL; fewer levels leave the
// valid region valid).  xch: the block's LDS exchange buffer.
template <typename real, int TL, int CI, int R, int W, int MODE>
__device__ __forceinline__ void tb_tile(const TbArgs<real> &p, int ti, int tj, int k0, int k1,
                                        int depth, real *xch)
{
    static_assert(TL >= 1 && TL <= JAC_MAX_DEPTH_DEV, "depth");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const AxisTile xi = axis_tile(ti, p.nx, 64 * CI, p.hi);
    const AxisTile xj = axis_tile(tj, p.ny, W * R, TL);
    const int kstart = max(k0 - depth, 0);
    const int nsteps = (k1 + depth) - kstart;  // steps kstart .. k1-1+depth

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
    int jrow[R];
    bool sh_j[R], ok_j[R];
    bool fix_j = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = xj.e + w * R + r;
        jrow[r] = j;
        rowoff[r] = (int64_t)min(max(j, 0), p.ny + 1) * p.sy;
        sh_j[r] = j == 0 || j == p.ny + 1;
        ok_j[r] = j >= xj.a && j < xj.b;
        fix_j = fix_j || sh_j[r];
    }

    // MODE_COMP: lanes 0..2 of wave 0 name the blocks of the same k chunk
    // whose inputs this block's output overwrites (the neighbours at -1 along
    // i, j and both for dir = +1, at +1 for dir = -1), and follow their
    // progress.
    int dep = -1, got = 0, pend = 0, self = 0;
    if constexpr (MODE == MODE_COMP) {
        const int tk = (k0 - 1) / p.kchunk;
        const int d = p.dir > 0 ? -1 : 1;
        const int a = ti + (lane == 1 ? 0 : d), b = tj + (lane == 0 ? 0 : d);
        if (w == 0 && lane < 3 && a >= 0 && a < p.nti && b >= 0 && b < p.ntj)
            dep = (tk * p.ntj + b) * p.nti + a;
        self = (tk * p.ntj + tj) * p.nti + ti;
    }

    // Plane k of an input array.  MODE_COMP: a halo plane that belongs to
    // another k chunk comes from the copy taken before the pass (its owner
    // may already have overwritten it); block boundary b (plane 1 + b*kchunk,
    // b >= 1) has planes [Kb - shift, Kb + shift] at copy slot b - 1.
    auto plane_base = [&](const real *src, int k) -> const real * {
        const int kc = min(max(k, 0), p.nz + 1);
        if constexpr (MODE == MODE_COMP) {
            if (kc >= 1 && kc <= p.nz && (kc < k0 || kc >= k1)) {
                const int kb = kc < k0 ? k0 : k1;
                const int64_t slot = (kb - 1) / p.kchunk - 1;
                return p.snap + (slot * (2 * p.shift + 1) + (kc - kb + p.shift)) * p.sz;
            }
        }
        return src + (int64_t)kc * p.sz;
    };
    auto load_plane = [&](const real *__restrict__ src, int k, real(&v)[R][CI]) {
        const real *plane = plane_base(src, k);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const real *row = plane + rowoff[r];
#pragma unroll
            for (int c = 0; c < CI; ++c)
                v[r][c] = row[ic[c]];
        }
    };

    // MODE_TRACE: record level s at the interior cells next to the shell (the
    // cells whose values the adjoint adds into the shell gradient).  Face
    // arrays of one level, F = 2(ny nz + nx nz + nx ny) values: i = 1 face
    // [k][j], i = nx face, j = 1 face [k][i], j = ny face, k = 1 face [j][i],
    // k = nz face.  Each value is written by the one block whose output
    // region holds the cell.
    auto trace_level = [&](int s, int plane, const real(&v)[R][CI]) {
        if constexpr (MODE == MODE_TRACE) {
            if (plane < k0 || plane >= k1)
                return;
            // One buffer resource per level and 32-bit byte offsets (the host
            // keeps a level of faces below 2^31 bytes): the row and plane
            // parts of an offset are wave-uniform, only the i part is per
            // lane, so the recording holds few registers across the loop.
            constexpr int E = (int)sizeof(real);
            const auto rs = plane_rsrc(p.trace + (int64_t)s * p.fstride, (int)(p.fstride * E));
            const int nyz = p.ny * p.nz, nxz = p.nx * p.nz, nxy = p.nx * p.ny;
            const int fj0 = 2 * nyz, fk0 = 2 * nyz + 2 * nxz;
            const bool klo = plane == 1, khi = plane == p.nz;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!ok_j[r])
                    continue;
                const int j = jrow[r];
                const bool jlo = j == 1, jhi = j == p.ny;
                if (klo || khi || jlo || jhi) {
                    const int kb = fk0 + (j - 1) * p.nx, jb = fj0 + (plane - 1) * p.nx;
#pragma unroll
                    for (int c = 0; c < CI; ++c) {
                        if (!ok_i[c])
                            continue;
                        const int i = ic[c] - 1;
                        if (klo)
                            plane_store(v[r][c], rs, (kb + i) * E);
                        if (khi)
                            plane_store(v[r][c], rs, (kb + nxy + i) * E);
                        if (jlo)
                            plane_store(v[r][c], rs, (jb + i) * E);
                        if (jhi)
                            plane_store(v[r][c], rs, (jb + nxz + i) * E);
                    }
                }
                if (fix_i) {
                    const int ib = (plane - 1) * p.ny + (j - 1);
#pragma unroll
                    for (int c = 0; c < CI; ++c) {
                        if (!ok_i[c])
                            continue;
                        if (ic[c] == 1)
                            plane_store(v[r][c], rs, ib * E);
                        if (ic[c] == p.nx)
                            plane_store(v[r][c], rs, (nyz + ib) * E);
                    }
                }
            }
        } else {
            (void)s;
            (void)plane;
            (void)v;
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
    if constexpr (MODE == MODE_COMP)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));  // the first plane is read (see step)

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
        if constexpr (MODE == MODE_COMP) {
            // Every load this wave issued has returned (plane k included):
            // the only vector memory operations issued after plane k's loads
            // are the previous step's R x CI output stores, and vmcnt counts
            // in issue order.  The last barrier followed the same wait of
            // every wave one step earlier, so all waves have read planes < k:
            // publish k.  (The counter store writes through to memory; issued
            // here, its latency overlaps this step.)
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(R * CI));
            if (threadIdx.x == 0 && k > kstart)
                __hip_atomic_store(p.prog + self, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // Wave 0 clears the next step's writes: before any wave overwrites
            // plane k + 1 - depth (after this step's barrier), the blocks that
            // read it must have read it, i.e. their progress > k + 1 - depth.
            // Polls are lazy: one answers for several steps while the
            // neighbours keep pace, and the next is issued the step before
            // its answer is needed, so its latency overlaps this step (a
            // counter poll reads memory, several microseconds under load).
            if (w == 0) {
                got = max(got, pend);
                const int wplane = k + 1 - depth;
                if (wplane >= k0 && wplane < k1) {
                    const int need = wplane + 1;
                    if (!__all(dep < 0 || got >= need)) {
                        int spins = 0;
                        for (;;) {
                            if (dep >= 0)
                                got = __hip_atomic_load(p.prog + dep, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                            if (__all(dep < 0 || got >= need))
                                break;
                            const int err = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                                p.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                            if (++spins > p.spin_limit || err) {
                                if (lane == 0)
                                    __hip_atomic_store(p.error, 1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    const bool stale = !__all(dep < 0 || got >= need + 1);
                    if (stale && dep >= 0)
                        pend = __hip_atomic_load(p.prog + dep, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
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
        trace_level(0, k, Qo[0]);

        // With two slabs, a level's edge rows go to LDS as soon as the level
        // is complete (every reader of this slab passed the previous
        // barrier), so the writes overlap the remaining levels.
        const int par = DBUF ? (k & 1) : 0;
        real *xcur = xch + par * XSLAB;
        auto publish = [&](int s) {
            if constexpr (DBUF) {
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    xcur[xidx(w, 0, s, c, lane)] = Qo[s][0][c];
                    xcur[xidx(w, 1, s, c, lane)] = Qo[s][R - 1][c];
                }
            } else {
                (void)s;
            }
        };
        if (depth > 0)
            publish(0);

        // ---- complete one plane per level, back to back; right after level s
        // completes, advance P[s-1] for the rows whose j-neighbours are in
        // registers.  The wave's first and last rows are finished after the
        // exchange; their Q values live in LDS (own slot, previous parity).
        const real *xold = xch + (DBUF ? (par ^ 1) : 0) * XSLAB;
#pragma unroll
        for (int s = 1; s <= TL; ++s) {
            if (s > depth)
                break;
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
            if (s < depth) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < CI; ++c)
                        Qo[s < TL ? s : 0][r][c] = o[r][c];
                trace_level(s, plane, Qo[s < TL ? s : 0]);
                publish(s < TL ? s : 0);
            } else if constexpr (MODE == MODE_BATCH) {
                if (plane >= k0 && plane < k1) {
                    real *dplane = p.dst + (int64_t)plane * p.sz;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (ok_j[r]) {
                            real *row = dplane + rowoff[r];
#pragma unroll
                            for (int c = 0; c < CI; ++c)
                                if (ok_i[c])
                                    __hip_atomic_store(&row[ic[c]], o[r][c], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                        }
                }
            } else {
                // The same R x CI stores on every step: cells outside the
                // valid region get the drop offset, and a plane outside
                // [k0, k1) a record count of 0.  vmcnt counts loads and stores
                // in issue order, so with a fixed store count the wait for the
                // next plane's loads at the end of the step no longer waits
                // for these stores (it did when they sat behind branches).
                const bool wr = plane >= k0 && plane < k1;
                const auto rs = plane_rsrc(p.dst + (int64_t)(wr ? plane : 0) * p.sz,
                                           wr ? (int)(p.sz * (int64_t)sizeof(real)) : 0);
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int c = 0; c < CI; ++c) {
                        const int off = (ok_j[r] && ok_i[c])
                                            ? (int)((rowoff[r] + ic[c]) * (int64_t)sizeof(real))
                                            : kDropOffset;
                        plane_store(o[r][c], rs, off);
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
        // The wave's own previous edge rows (the D terms of its edge rows' P)
        // are read before the barrier, so that only the neighbours' rows are
        // read after it.  (With one buffer they must be: the slot is about to
        // be overwritten.)
        real dold[TL][2][CI];
#pragma unroll
        for (int s = 0; s < TL; ++s)
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                dold[s][0][c] = xold[xidx(w, 0, s, c, lane)];
                dold[s][1][c] = xold[xidx(w, 1, s, c, lane)];
            }
        if constexpr (!DBUF)
            __syncthreads();
        // the first term of the edge rows' P (west + east, from registers
        // and DPP) before the barrier too: after it only the terms from the
        // neighbouring waves remain
        real we[TL][2][CI];
#pragma unroll
        for (int s = 0; s < TL; ++s) {
            if (s >= depth)
                break;
            real west[CI], east[CI];
            neighbours_i(Qo[s][0], west, east);
#pragma unroll
            for (int c = 0; c < CI; ++c)
                we[s][0][c] = west[c] + east[c];
            if constexpr (R > 1) {
                neighbours_i(Qo[s][R - 1], west, east);
#pragma unroll
                for (int c = 0; c < CI; ++c)
                    we[s][1][c] = west[c] + east[c];
            }
        }
        if constexpr (!DBUF) {
#pragma unroll
            for (int s = 0; s < TL; ++s)
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    if (s < depth) {
                        xcur[xidx(w, 0, s, c, lane)] = Qo[s][0][c];
                        xcur[xidx(w, 1, s, c, lane)] = Qo[s][R - 1][c];
                    }
                }
        }
        __syncthreads();
        auto dprev = [&](int side, int s, int c) -> real { return dold[s][side][c]; };
#pragma unroll
        for (int s = 0; s < TL; ++s) {
            if (s >= depth)
                break;
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                const real sn = xcur[xidx(wa, 1, s, c, lane)];
                const real north = R > 1 ? Qo[s][R > 1 ? 1 : 0][c] : xcur[xidx(wb, 0, s, c, lane)];
                real q = we[s][0][c];
                q = q + sn;
                q = q + north;
                P[s][0][c] = q + dprev(0, s, c);
            }
            if constexpr (R > 1) {
#pragma unroll
                for (int c = 0; c < CI; ++c) {
                    const real nn = xcur[xidx(wb, 0, s, c, lane)];
                    real q = we[s][1][c];
                    q = q + Qo[s][R - 2][c];
                    q = q + nn;
                    P[s][R - 1][c] = q + dprev(1, s, c);
                }
            }
        }
    };

    // A wave all of whose rows lie past the shell row ny+1 (the tail of the
    // last block along j) computes nothing any output needs: no live row
    // reads its rows (a live wave's last row next to it is then the shell row
    // or past it).  It only takes part in the step's barriers, so its SIMD's
    // issue slots go to the other waves (batches of small grids leave up to
    // a third of the waves dead).  Wave 0 is never dead: a block starts at or
    // below row ny.
    // (Two loops rather than a test inside one: a path around the step
    // inside the loop makes the compiler keep both sets of carried values.)
    const bool dead = xj.e + w * R > p.ny + 1;
    if (dead) {
        for (int n = 0; n < nsteps; ++n) {
            if constexpr (!DBUF)
                __syncthreads();  // the barrier before a live step overwrites its slab
            __syncthreads();      // the barrier after the slab is written
        }
    }
    for (int n = 0; n < (dead ? 0 : nsteps); ++n) {
        step(kstart + n, QA, QB, CA, CB);
#pragma unroll
        for (int s = 0; s < TL; ++s)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < CI; ++c)
                    QA[s][r][c] = QB[s][r][c];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < CI; ++c)
                CA[r][c] = CB[r][c];
    }
    if constexpr (MODE == MODE_COMP) {
        // done: every plane this block reads has been read
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(p.prog + self, 1 << 30, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One pass over a whole grid: workgroup (ti, tj, tk) streams output planes
// [1 + tk*kchunk, 1 + (tk+1)*kchunk) of block column (ti, tj).  The k chunk
// is the slowest index, so the workgroups that run at the same time stream
// the same few planes of the grid: contiguous memory, which the DRAM serves
// much faster than planes scattered over the grid.
template <typename real, int TL, int CI, int R, int W, int MODE>
__global__ __launch_bounds__(64 * W) void tblock_kernel(TbArgs<real> p)
{
    extern __shared__ unsigned char smem_raw[];
    real *xch = reinterpret_cast<real *>(smem_raw);  // [parity][W][2][TL][CI][64]
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int ti = bid % p.nti;
    const int tj = (bid / p.nti) % p.ntj;
    const int tk = bid / (p.nti * p.ntj);
    const int k0 = 1 + tk * p.kchunk;
    tb_tile<real, TL, CI, R, W, MODE>(p, ti, tj, k0, min(k0 + p.kchunk, p.nz + 1), TL, xch);
}

// One pass of the compressed single grid (Sect. 1.3): src and dst are two
// frames of one array, dst shifted by (-shift, -shift, 0) cells against src
// (dir = +1) or by (+shift, +shift, 0) (dir = -1), shift >= the halo.  A
// block then overwrites only inputs of itself and of its neighbours at -1
// along i, j or both (dir = +1; at +1 for dir = -1) in the same k chunk:
// every other block reads none of the cells it writes, and halo planes of
// other k chunks come from copies (plane_base).  So each block waits, per
// plane, until those three neighbours have read the plane it overwrites
// (write after read; no block reads what another writes in the same pass).
// Workgroups take tickets in order and a ticket's blocks depend only on
// blocks of earlier tickets, held by running workgroups, so waits end.
template <typename real, int TL, int CI, int R, int W>
__global__ __launch_bounds__(64 * W) void compressed_kernel(TbArgs<real> p)
{
    // dynamic LDS follows the static ticket_s: align it for 8-byte accesses
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    real *xch = reinterpret_cast<real *>(smem_raw);
    __shared__ int ticket_s;
    if (threadIdx.x == 0)
        ticket_s = atomicAdd(p.ticket, 1);
    __syncthreads();
    const int m = ticket_s;
    const int nkc = (p.nz + p.kchunk - 1) / p.kchunk;
    if (m >= p.nti * p.ntj * nkc)
        return;  // more workgroups than blocks: nothing to do
    int ti = m % p.nti, tj = (m / p.nti) % p.ntj;
    const int tk = m / (p.nti * p.ntj);
    if (p.dir < 0) {
        ti = p.nti - 1 - ti;
        tj = p.ntj - 1 - tj;
    }
    const int k0 = 1 + tk * p.kchunk;
    tb_tile<real, TL, CI, R, W, MODE_COMP>(p, ti, tj, k0, min(k0 + p.kchunk, p.nz + 1), TL, xch);
}

// Batched pass over many grids (items of the plan).  In persistent mode each
// workgroup pops items in order; an item of pass p first waits until every
// neighbouring block (the 3 x 3 x 3 blocks around it, itself included) of
// the same grid has finished pass p-1.  That one lower-bound condition both
// guarantees that the level-0 data it reads are written (read after write)
// and that the neighbours have finished reading the buffer it overwrites
// (write after read): the lower-bound half of the relaxed synchronisation of
// Sect. 1.3 (Eq. 3), with a per-block counter in place of a per-thread one.
// Items are handed out in pass order and a block waits only on items handed
// out before its own, all held by running blocks, so the waits always end.
// FIXED: every item of the launch has depth TL (all grids run T a multiple of
// t); the depth is then a compile-time constant, which saves registers.
template <typename real, int TL, int CI, int R, int W, bool FIXED>
__global__ __launch_bounds__(64 * W) void batched_kernel(BatchLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    real *xch = reinterpret_cast<real *>(smem_raw);
    __shared__ int item_s, stop_s;
    int it = L.begin + (int)blockIdx.x;
    for (;;) {
        if (L.persistent) {
            // thread 0 decides for the whole workgroup: the next item, and
            // whether a wait somewhere gave up (then stop taking work)
            if (threadIdx.x == 0) {
                item_s = L.begin + atomicAdd(&L.counters[0], 1);
                stop_s = __hip_atomic_load(L.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            it = item_s;
            const int stop = stop_s;
            __syncthreads();
            if (stop)
                break;
        }
        if (it >= L.end)
            break;
        const BatchItem m = L.items[it];
        // stress runs only: hold the item back before it reads or writes
        // anything (the waits of the items that need it absorb the delay)
        for (int s = 0; s < m.delay; ++s)
            __builtin_amdgcn_s_sleep(127);
        const BatchGrid G = L.grids[m.grid];
        const int ti = m.tile % G.nti;
        const int tj = (m.tile / G.nti) % G.ntj;
        const int tk = m.tile / (G.nti * G.ntj);
        int *cnt = L.counters + 1 + G.counter_off;
        if (L.persistent && (m.pass > 0 || G.team > 0)) {
            // wave 0 polls every counter the item waits on at once, until
            // every lane sees its condition hold:
            //  * lanes 0..26: the block at offset (n % 3, n / 3 % 3, n / 9) - 1
            //    has finished the previous pass (the data the item reads);
            //  * pipelined runs (Eq. 3, distances in k chunks beyond the
            //    one-chunk halo): lane 27, the previous pass has finished the
            //    same block column's chunk tk + dl (+ dt at a segment's front,
            //    the team delay); lane 28, the next pass has finished chunk
            //    tk - du - 2 (the upper bound; not at a segment's rear pass)
            if (threadIdx.x < 64) {
                const int n = threadIdx.x;
                int a = ti, b = tj, c = tk, need = m.pass;
                bool mine = false;
                if (n < 27) {
                    a = ti + n % 3 - 1;
                    b = tj + n / 3 % 3 - 1;
                    c = tk + n / 9 - 1;
                    mine = m.pass > 0;
                } else if (n == 27 && G.team > 0 && m.pass > 0) {
                    c = min(tk + G.dl + (m.pass % G.team == 0 ? G.dt : 0), G.nkc - 1);
                    mine = true;
                } else if (n == 28 && G.team > 0 && G.du > 0 && m.pass % G.team != G.team - 1 &&
                           m.pass + 1 < G.passes) {
                    c = tk - G.du - 2;
                    need = m.pass + 2;
                    mine = c >= 0;
                }
                mine = mine && a >= 0 && a < G.nti && b >= 0 && b < G.ntj && c >= 0 && c < G.nkc;
                const int *q = cnt + (mine ? (c * G.ntj + b) * G.nti + a : 0);
                // bounded wait (seconds): a wait that cannot end raises the
                // error flag instead of hanging; every decision is wave-uniform
                int spins = 0;
                for (;;) {
                    const bool ok =
                        !mine || __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
                    if (__all(ok))
                        break;
                    __builtin_amdgcn_s_sleep(2);
                    const int err = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(L.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (++spins > L.spin_limit || err) {
                        if (n == 0)
                            __hip_atomic_store(L.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        TbArgs<real> p;
        p.src = (const real *)((m.pass % 2 == 0) ? G.a : (const void *)G.b);
        p.dst = (real *)((m.pass % 2 == 0) ? G.b : (void *)G.a);
        p.rhs = nullptr;
        p.trace = nullptr;
        p.sy = G.sy;
        p.sz = G.sz;
        p.nx = G.nx;
        p.ny = G.ny;
        p.nz = G.nz;
        p.nti = G.nti;
        p.ntj = G.ntj;
        p.hi = G.hi;
        p.fstride = 0;
        p.kchunk = G.kchunk;
        const int depth = G.T / G.passes + (m.pass < G.T % G.passes ? 1 : 0);
        const int k0 = 1 + tk * G.kchunk;
        tb_tile<real, TL, CI, R, W, MODE_BATCH>(p, ti, tj, k0, min(k0 + G.kchunk, G.nz + 1),
                                                FIXED ? TL : depth, xch);
        if (!L.persistent)
            break;
        // Publish.  The item's output stores are agent-scope, so they write
        // through this XCD's L2, and every wave waits until its own stores
        // have completed (vmcnt 0) before the barrier; thread 0 then bumps
        // the counter with an agent-scope release store, which pairs with the
        // consumer's agent-scope acquire fence: every store of the item
        // happens before the barrier, the barrier before the release, so the
        // consumer that sees the counter also sees the data, by the memory
        // model and not only by how the hardware orders write-through stores.
        // (With the data already written through, the release has little
        // left to write back.)
        __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(cnt + m.tile, m.pass + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename real, int TL, int CI, int R, int W>
static KernInfo batch_info_one(int fixed)
{
    const void *fn = fixed ? (const void *)batched_kernel<real, TL, CI, R, W, true>
                           : (const void *)batched_kernel<real, TL, CI, R, W, false>;
    return KernInfo{fn, xch_bytes<real, TL, CI, W>(), 64 * W};
}

template <typename real, int CI, int R, int W>
static KernInfo batch_info_depth(int depth, int fixed)
{
    switch (depth) {
    case 1: return batch_info_one<real, 1, CI, R, W>(fixed);
    case 2: return batch_info_one<real, 2, CI, R, W>(fixed);
    case 3: return batch_info_one<real, 3, CI, R, W>(fixed);
    case 4: return batch_info_one<real, 4, CI, R, W>(fixed);
    case 5: return batch_info_one<real, 5, CI, R, W>(fixed);
    case 6: return batch_info_one<real, 6, CI, R, W>(fixed);
    case 7: return batch_info_one<real, 7, CI, R, W>(fixed);
    case 8: return batch_info_one<real, 8, CI, R, W>(fixed);
    default: return KernInfo{nullptr, 0, 0};
    }
}

template <typename real>
static KernInfo batch_info(int cfg, int depth, int fixed)
{
#define JAC_CFG(ID, CI, R, W) \
    case ID: return batch_info_depth<real, CI, R, W>(depth, fixed);
    switch (cfg) {
        JAC_TILE_MENU(JAC_CFG)
    default: return KernInfo{nullptr, 0, 0};
    }
#undef JAC_CFG
}

// Compressed-grid instances exist for 64-wide blocks (CI = 1) only.
template <typename real, int TL, int CI, int R, int W>
static KernInfo comp_info_one()
{
    if constexpr (CI == 1)
        return KernInfo{(const void *)compressed_kernel<real, TL, CI, R, W>,
                        xch_bytes<real, TL, CI, W>(), 64 * W};
    else
        return KernInfo{nullptr, 0, 0};
}

template <typename real, int CI, int R, int W>
static KernInfo comp_info_depth(int depth)
{
    switch (depth) {
    case 1: return comp_info_one<real, 1, CI, R, W>();
    case 2: return comp_info_one<real, 2, CI, R, W>();
    case 3: return comp_info_one<real, 3, CI, R, W>();
    case 4: return comp_info_one<real, 4, CI, R, W>();
    case 5: return comp_info_one<real, 5, CI, R, W>();
    case 6: return comp_info_one<real, 6, CI, R, W>();
    case 7: return comp_info_one<real, 7, CI, R, W>();
    case 8: return comp_info_one<real, 8, CI, R, W>();
    default: return KernInfo{nullptr, 0, 0};
    }
}

template <typename real>
static KernInfo comp_info(int cfg, int depth)
{
#define JAC_CFG(ID, CI, R, W) \
    case ID: return comp_info_depth<real, CI, R, W>(depth);
    switch (cfg) {
        JAC_TILE_MENU(JAC_CFG)
    default: return KernInfo{nullptr, 0, 0};
    }
#undef JAC_CFG
}

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

template <typename real, int MODE>
static KernInfo tb_info_mode(int cfg, int depth)
{
#define JAC_CFG(ID, CI, R, W) \
    case ID: return tb_info_depth<real, CI, R, W, MODE>(depth);
    switch (cfg) {
        JAC_TILE_MENU(JAC_CFG)
    default: return KernInfo{nullptr, 0, 0};
    }
#undef JAC_CFG
}

}  // namespace jac
