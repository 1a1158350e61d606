/*
 * lbm.h -- the D3Q19 lattice Boltzmann steps of libjacobi.so (gfx950).
 *
 * The paper treats the Jacobi sweep as the prototype of the lattice
 * Boltzmann method (LBM) and names a temporally blocked LBM solver as the
 * goal of the work (Sect. 1.1, Sect. 3).  It prints no LBM equations; this
 * entry point implements the textbook single-relaxation-time (BGK) scheme on
 * the D3Q19 lattice:
 *   velocities  c_0 = (0,0,0); c_1..c_6 = (+-1,0,0), (0,+-1,0), (0,0,+-1) in
 *               that order; c_7..c_18 = (1,1,0), (-1,-1,0), (1,-1,0),
 *               (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1),
 *               (0,-1,-1), (0,1,-1), (0,-1,1);
 *   weights     w_0 = 1/3, w_1..6 = 1/18, w_7..18 = 1/36;
 *   one step    g_i = f_i(x - c_i, t)  (streaming, periodic box),
 *               rho = sum_i g_i, rho u = sum_i c_i g_i,
 *               feq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u),
 *               f_i(x, t+1) = g_i - omega (g_i - feq_i).
 * Arithmetic order, fixed so that FP64 results are reproducible bit for bit:
 * the density and momentum sums run over the populations in index order
 * starting from 0; c_i.u adds the nonzero components of c_i in x, y, z order
 * starting from 0; feq_i = (w_i rho) (((1 + 3 cu) + 9/2 (cu cu)) - 3/2 usq)
 * with usq = (ux ux + uy uy) + uz uz; divisions are IEEE.  FP32 uses the same
 * order in single precision.
 *
 * Layout: 19 arrays of n = nx*ny*nz values one after another (population i
 * at base + i*n), cell (x, y, z) at x + nx*(y + ny*z): device pointers owned
 * by the caller.  Errors and jacobi_last_error() are those of jacobi.h.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#include "jacobi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_grid {
    int64_t nx, ny, nz;
} lbm_grid_t;

/* T steps of D3Q19 BGK on a periodic box.  f holds the populations of step 0;
 * f_tmp is a second buffer of the same size (19*n values of dtype; contents
 * ignored, not overlapping f).  Steps write f and f_tmp in turn: on return
 * *out_idx says which holds step T (0 = f, 1 = f_tmp; T mod 2).  dtype:
 * JAC_F32 or JAC_F64.  nx, ny, nz >= 1, nx*ny*nz*19 values addressable with
 * 63-bit offsets, ny*ceil(nx/64) < 2^31 / 4 and nz <= 65535 (grid limits);
 * omega the relaxation rate (finite; 0 < omega < 2 for a stable flow, not
 * checked).  T >= 0 (T = 0 enqueues nothing).  Argument checks happen before
 * any HIP call; the call enqueues on `stream` and returns without
 * synchronising. */
int lbm_d3q19_steps(int dtype, const lbm_grid_t *g, void *f, void *f_tmp, double omega, int T,
                    void *stream, int *out_idx);

/* The same T steps with temporal blocking at depth 2 (Sect. 1.1: two time
 * steps per pass over memory): each pass reads the populations once and
 * writes them once for two steps, keeping the intermediate step's
 * populations on chip.  A workgroup computes the intermediate step on a
 * region of 32 x 8 cells (x, y; 32 x 16 in FP32) and the second step on the
 * cells one inside it (30 x 6, or 30 x 14), streaming z chunks of kchunk
 * planes (0 = library choice: 12 in FP64, 4 in FP32, or nz if smaller;
 * 1..65535).  An odd T ends with one plain step.  Every
 * cell runs the same arithmetic as lbm_d3q19_steps, so the results are
 * bitwise those of lbm_d3q19_steps (and of the plain sequential scheme
 * above).  Buffers alternate once per pass: *out_idx = (number of passes
 * plus the plain step) mod 2 names the one holding step T.  Other arguments
 * and errors as for lbm_d3q19_steps; ceil(ny/6) (FP32: ceil(ny/14)) must not
 * exceed 65535. */
int lbm_d3q19_blocked(int dtype, const lbm_grid_t *g, void *f, void *f_tmp, double omega, int T,
                      int kchunk, void *stream, int *out_idx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
