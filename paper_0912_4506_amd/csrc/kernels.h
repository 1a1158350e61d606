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
    X(5, 2, 2, 8)

namespace jac {

enum { MODE_PLAIN = 0, MODE_RHS = 1, MODE_TRACE = 2 };

struct GridArgs {
    int64_t nx, ny, nz, sy, sz;
};

struct PlainArgs {
    int nx, ny, nz, kchunk;
    int64_t sy, sz;
};

template <typename real>
struct TbArgs {
    const real *src;
    real *dst;
    const real *rhs;
    real *trace;
    int64_t sy, sz;
    int nx, ny, nz;
    int nti, ntj, nkc;  // blocks along i, j, k
    int hi;             // i-halo (>= depth; even when CI is even, for alignment)
    int kchunk;         // output planes per block along k
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
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

// Resident workgroups per CU of a tblock instance (0 when it cannot launch).
int tblock_occupancy(int dtype, int cfg, int depth, int mode);

}  // namespace jac
