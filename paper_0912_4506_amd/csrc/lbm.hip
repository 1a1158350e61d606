// D3Q19 lattice Boltzmann time steps (gfx950): the stencil method the paper
// takes the Jacobi sweep as a prototype of (Sect. 1.1) and names as the
// target of temporal blocking (Sect. 3).  Single-relaxation-time (BGK)
// collision, periodic box, fused streaming ("pull") and collision: every cell
// gathers population i from x - c_i, computes density and velocity, and
// relaxes towards the second-order equilibrium
//     feq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u).
// Arithmetic order (fixed, so FP64 results are reproducible bit for bit):
// density and momentum sum the populations in index order starting from 0,
// c_i.u adds the nonzero components in x, y, z order starting from 0,
// feq_i = (w_i rho) (((1 + 3 cu) + 9/2 (cu cu)) - 3/2 usq) with
// usq = (ux ux + uy uy) + uz uz, and f_i' = g_i - omega (g_i - feq_i).
//
// One thread per cell: 19 loads (each population from its own array at a
// shifted position, so every stored value is read exactly once per step),
// about 200 flops, 19 stores.  Algorithmic traffic 2 * 19 * sizeof(real)
// bytes per lattice-site update: the kernel is HBM-bound by a wide margin.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace jac {

namespace {

// The D3Q19 velocity set: rest, six face neighbours, twelve edge neighbours;
// populations 2m-1 and 2m point in opposite directions.
constexpr int kQ = 19;
constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <typename real>
__device__ __forceinline__ real lbm_weight(int i)
{
    return i == 0 ? real(1) / real(3) : (i <= 6 ? real(1) / real(18) : real(1) / real(36));
}

// sum of the components a velocity component c selects: +v, -v or nothing
template <typename real>
__device__ __forceinline__ real add_component(real acc, int c, real v)
{
    return c == 1 ? acc + v : (c == -1 ? acc - v : acc);
}

// One cell's collision: g holds the 19 populations gathered by streaming;
// out receives the relaxed populations.  Both kernels run this code, so a
// cell's update is the same instruction sequence in either.
template <typename real>
__device__ __forceinline__ void collide(const real (&g)[kQ], real omega, real (&out)[kQ])
{
    real rho = real(0), jx = real(0), jy = real(0), jz = real(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        rho = rho + g[i];
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        jx = add_component(jx, kCx[i], g[i]);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        jy = add_component(jy, kCy[i], g[i]);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        jz = add_component(jz, kCz[i], g[i]);
    const real ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const real usq = (ux * ux + uy * uy) + uz * uz;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        real cu = real(0);
        cu = add_component(cu, kCx[i], ux);
        cu = add_component(cu, kCy[i], uy);
        cu = add_component(cu, kCz[i], uz);
        const real t = ((real(1) + real(3) * cu) + real(4.5) * (cu * cu)) - real(1.5) * usq;
        const real feq = (lbm_weight<real>(i) * rho) * t;
        out[i] = g[i] - omega * (g[i] - feq);
    }
}

__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

constexpr int kLbmX = 64, kLbmY = 4;  // cells of a block along x and y

template <typename real>
__global__ __launch_bounds__(kLbmX * kLbmY) void lbm_d3q19_kernel(const real *__restrict__ f,
                                                                real *__restrict__ out,
                                                                LbmArgs p)
{
    int bx, by, bz;
    remapped_block(bx, by, bz);
    const int x = bx * kLbmX + (int)(threadIdx.x % kLbmX);
    const int y = by * kLbmY + (int)(threadIdx.x / kLbmX);
    const int z = bz;
    if (x >= p.nx || y >= p.ny)
        return;
    // neighbour coordinates on the periodic box: index 0, 1, 2 = c - 1, c, c + 1
    const int xs[3] = {x == 0 ? p.nx - 1 : x - 1, x, x + 1 == p.nx ? 0 : x + 1};
    const int ys[3] = {y == 0 ? p.ny - 1 : y - 1, y, y + 1 == p.ny ? 0 : y + 1};
    const int zs[3] = {z == 0 ? p.nz - 1 : z - 1, z, z + 1 == p.nz ? 0 : z + 1};

    // streaming: population i arrives from x - c_i
    real g[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int64_t src = (int64_t)xs[1 - kCx[i]] +
                            (int64_t)p.nx * ((int64_t)ys[1 - kCy[i]] + (int64_t)p.ny * zs[1 - kCz[i]]);
        g[i] = f[(int64_t)i * p.n + src];
    }
    real o[kQ];
    collide<real>(g, (real)p.omega, o);
    const int64_t cell = (int64_t)x + (int64_t)p.nx * ((int64_t)y + (int64_t)p.ny * z);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        out[(int64_t)i * p.n + cell] = o[i];
}

// ---------------------------------------------------------- depth 2 pass --
// Two time steps per pass over memory (temporal blocking, Sect. 1.1, applied
// to the D3Q19 stream-collide step).  A workgroup owns a level-1 region of
// X x Y cells (one per thread; Lbm2Shape) and the output tile one cell
// inside it, and streams a chunk of z planes.  At stream step s
// it computes level 1 (step t+1) of plane zs = z0 - 1 + s on the whole
// region, pulling level 0 straight from memory, then level 2 (step t+2) of
// plane zs - 1 on the tile, pulling level 1 from LDS.  Level 2 of plane z
// pulls the populations with c_z = -1 from level-1 plane z + 1 (the one just
// computed), those with c_z = 0 from plane z, those with c_z = +1 from plane
// z - 1; so LDS keeps one plane of the first group, two of the second and
// three of the third (38 population planes of the region, not 57).  The
// level-0 pulls of the next step are issued before the level-2 work of this
// one.  Algorithmic traffic: one read and one write of 19 values per cell per
// two steps.
// the populations by z velocity: group 0 (c_z = -1), 1 (c_z = 0), 2 (c_z = +1)
constexpr int kGroup[kQ] = {1, 1, 1, 1, 1, 2, 0, 1, 1, 1, 1, 2, 0, 0, 2, 2, 0, 0, 2};
constexpr int kGroupIdx[kQ] = {0, 1, 2, 3, 4, 0, 0, 5, 6, 7, 8, 1, 1, 2, 2, 3, 3, 4, 4};
constexpr int kGroupSize[3] = {5, 9, 5};
constexpr int kGroupSlots[3] = {1, 2, 3};
// offsets (in population planes) of each group's slots in LDS
constexpr int kGroupBase[3] = {0, 5, 5 + 2 * 9};
constexpr int kLbm2Planes = 5 + 2 * 9 + 3 * 5;  // 38

template <typename real>
struct Lbm2Shape {
    static constexpr int X = lbm2_region_x(sizeof(real)), Y = lbm2_region_y(sizeof(real));
    static constexpr int Cells = X * Y;
    static constexpr size_t lds = (size_t)kLbm2Planes * Cells * sizeof(real);
};

template <typename real>
__global__ __launch_bounds__(Lbm2Shape<real>::Cells) void lbm_d3q19_x2_kernel(
    const real *__restrict__ f, real *__restrict__ out, LbmArgs p, int kchunk)
{
    constexpr int kLbm2X = Lbm2Shape<real>::X, kLbm2Y = Lbm2Shape<real>::Y;
    constexpr int kLbm2Cells = Lbm2Shape<real>::Cells;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    real *lds = reinterpret_cast<real *>(smem_raw);
    int tx, ty, tz;
    remapped_block(tx, ty, tz);
    const int lx = (int)threadIdx.x % kLbm2X, ly = (int)threadIdx.x / kLbm2X;
    const int c = (int)threadIdx.x;
    // region cell of this thread (unwrapped x0 + lx, y0 + ly) and its box cell
    const int ux = tx * (kLbm2X - 2) - 1 + lx, uy = ty * (kLbm2Y - 2) - 1 + ly;
    const int x = wrap(ux, p.nx), y = wrap(uy, p.ny);
    const int xs[3] = {wrap(x - 1, p.nx), x, wrap(x + 1, p.nx)};
    const int ys[3] = {wrap(y - 1, p.ny), y, wrap(y + 1, p.ny)};
    // output cell: inside the tile and inside the box
    const bool outc = lx >= 1 && lx < kLbm2X - 1 && ly >= 1 && ly < kLbm2Y - 1 && ux < p.nx &&
                      uy < p.ny;
    const int z0 = tz * kchunk, z1 = min(z0 + kchunk, p.nz);
    const real omega = (real)p.omega;

    // level-0 pulls of level-1 plane zs into v
    auto gather0 = [&](int zs, real(&v)[kQ]) {
        const int zc = wrap(zs, p.nz);
        const int zz[3] = {wrap(zc - 1, p.nz), zc, wrap(zc + 1, p.nz)};
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int64_t src = (int64_t)xs[1 - kCx[i]] +
                                (int64_t)p.nx * ((int64_t)ys[1 - kCy[i]] + (int64_t)p.ny * zz[1 - kCz[i]]);
            v[i] = f[(int64_t)i * p.n + src];
        }
    };
    // LDS slot of population i of the level-1 plane computed at step s
    auto slot = [&](int i, int s) -> real * {
        const int g = kGroup[i];
        const int k = s % kGroupSlots[g];
        return lds + (size_t)(kGroupBase[g] + k * kGroupSize[g] + kGroupIdx[i]) * kLbm2Cells;
    };

    // One stream step s: level 1 of plane z0 - 1 + s from the level-0 pulls
    // in cur, then (once three level-1 planes exist) level 2 of plane
    // z0 + s - 2.  The pulls of step s + 2 go into cur as soon as level 1 has
    // used it, so each step's loads have two steps to arrive (the loop runs
    // two steps per iteration with the two register sets swapping roles).
    const int nsteps = z1 - z0 + 2;  // level-1 planes z0-1 .. z1
    auto step = [&](int s, real(&cur)[kQ]) {
        real f1[kQ];
        collide<real>(cur, omega, f1);
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            slot(i, s)[c] = f1[i];
        __syncthreads();
        if (s + 2 < nsteps)
            gather0(z0 + s + 1, cur);
        if (s >= 2 && outc) {
            // level 2 of plane zo = zs - 1 from level-1 planes zo+1 (step s), zo (s-1), zo-1 (s-2)
            real g[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int from = (lx - kCx[i]) + kLbm2X * (ly - kCy[i]);
                g[i] = slot(i, s - 1 - kCz[i])[from];
            }
            real o[kQ];
            collide<real>(g, omega, o);
            const int zo = z0 + s - 2;
            const int64_t cell = (int64_t)ux + (int64_t)p.nx * ((int64_t)uy + (int64_t)p.ny * zo);
#pragma unroll
            for (int i = 0; i < kQ; ++i)
                out[(int64_t)i * p.n + cell] = o[i];
        }
        __syncthreads();  // the next step overwrites slots read here
    };
    real ga[kQ], gb[kQ];
    gather0(z0 - 1, ga);
    gather0(z0, gb);  // nsteps >= 3
    int s = 0;
    for (; s + 1 < nsteps; s += 2) {
        step(s, ga);
        step(s + 1, gb);
    }
    if (s < nsteps)
        step(s, ga);
}

}  // namespace

template <typename real>
hipError_t launch_lbm_d3q19(const real *f, real *out, const LbmArgs &p, hipStream_t st)
{
    const dim3 grid((unsigned)((p.nx + kLbmX - 1) / kLbmX), (unsigned)((p.ny + kLbmY - 1) / kLbmY),
                    (unsigned)p.nz);
    hipLaunchKernelGGL(lbm_d3q19_kernel<real>, grid, dim3(kLbmX * kLbmY), 0, st, f, out, p);
    return hipGetLastError();
}

template hipError_t launch_lbm_d3q19<float>(const float *, float *, const LbmArgs &, hipStream_t);
template hipError_t launch_lbm_d3q19<double>(const double *, double *, const LbmArgs &, hipStream_t);

template <typename real>
hipError_t launch_lbm_d3q19_x2(const real *f, real *out, const LbmArgs &p, int kchunk, hipStream_t st)
{
    constexpr int kLbm2X = Lbm2Shape<real>::X, kLbm2Y = Lbm2Shape<real>::Y;
    const size_t lds = Lbm2Shape<real>::lds;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)lbm_d3q19_x2_kernel<real>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    const dim3 grid((unsigned)((p.nx + kLbm2X - 3) / (kLbm2X - 2)),
                    (unsigned)((p.ny + kLbm2Y - 3) / (kLbm2Y - 2)),
                    (unsigned)((p.nz + kchunk - 1) / kchunk));
    hipLaunchKernelGGL(lbm_d3q19_x2_kernel<real>, grid, dim3(Lbm2Shape<real>::Cells), lds, st, f, out,
                       p, kchunk);
    return hipGetLastError();
}

template hipError_t launch_lbm_d3q19_x2<float>(const float *, float *, const LbmArgs &, int, hipStream_t);
template hipError_t launch_lbm_d3q19_x2<double>(const double *, double *, const LbmArgs &, int,
                                                hipStream_t);

}  // namespace jac
