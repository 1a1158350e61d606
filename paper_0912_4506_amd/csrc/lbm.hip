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

    // moments
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
    const real omega = (real)p.omega;

    // collision, and the store of the new populations at x
    const int64_t cell = (int64_t)x + (int64_t)p.nx * ((int64_t)y + (int64_t)p.ny * z);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        real cu = real(0);
        cu = add_component(cu, kCx[i], ux);
        cu = add_component(cu, kCy[i], uy);
        cu = add_component(cu, kCz[i], uz);
        const real t = ((real(1) + real(3) * cu) + real(4.5) * (cu * cu)) - real(1.5) * usq;
        const real feq = (lbm_weight<real>(i) * rho) * t;
        out[(int64_t)i * p.n + cell] = g[i] - omega * (g[i] - feq);
    }
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

}  // namespace jac
