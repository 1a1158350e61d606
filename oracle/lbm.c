/*
 * CPU oracle for the D3Q19 lattice Boltzmann workload -- TEST INFRASTRUCTURE
 * ONLY.
 *
 * The paper treats the Jacobi sweep as the prototype of the lattice Boltzmann
 * method (LBM) and names a temporally blocked LBM solver as the goal it is
 * working towards (Sect. 1.1, Sect. 3).  It prints no LBM equations, so this
 * file follows the textbook single-relaxation-time (BGK) scheme on the D3Q19
 * lattice: 19 populations per cell, one per velocity of the set below, with
 * the usual weights 1/3 (rest), 1/18 (six face neighbours) and 1/36 (twelve
 * edge neighbours), and the second-order equilibrium
 *     feq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u).
 * One time step: every cell gathers population i from its neighbour at
 * x - c_i (streaming, "pull") and relaxes the gathered set towards the
 * equilibrium of its own moments with rate omega (collision):
 *     rho = sum_i g_i,  rho u = sum_i c_i g_i,
 *     f_i(x, t+1) = g_i - omega (g_i - feq_i(rho, u)),
 * with g_i = f_i(x - c_i, t).  The box is periodic on every axis.
 *
 * Arithmetic: IEEE binary64 in the order written (built with
 * -ffp-contract=off, no -ffast-math): the density and momentum sums run over
 * the populations in index order from 0, a population's c.u sums the nonzero
 * velocity components in x, y, z order from 0, and
 *     feq_i = (w_i * rho) * (((1 + 3 cu) + 9/2 (cu cu)) - 3/2 usq),
 *     usq   = (ux ux + uy uy) + uz uz.
 *
 * Layout: 19 arrays of n = nx*ny*nz values one after another, population i
 * at f + i*n, cell (x, y, z) at x + nx*(y + ny*z).
 *
 * Nothing here is shared with the GPU library.
 */
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* Velocity set: the rest velocity, the six face neighbours, the twelve edge
 * neighbours; populations 2m-1 and 2m point in opposite directions. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

static double weight(int i)
{
    if (i == 0)
        return 1.0 / 3.0;
    return i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0;
}

/* The velocity set (57 ints, c_i at 3i) and the weights (19 doubles). */
void oracle_lbm_lattice(int *c, double *w)
{
    for (int i = 0; i < Q; i++) {
        for (int a = 0; a < 3; a++)
            c[3 * i + a] = CV[i][a];
        w[i] = weight(i);
    }
}

/* c_i . u: the nonzero components of c_i in x, y, z order, added to 0. */
static double c_dot_u(int i, const double u[3])
{
    double cu = 0.0;
    for (int a = 0; a < 3; a++) {
        if (CV[i][a] == 1)
            cu = cu + u[a];
        else if (CV[i][a] == -1)
            cu = cu - u[a];
    }
    return cu;
}

/* The 19 equilibrium populations of density rho and velocity u. */
void oracle_lbm_equilibrium(double rho, double ux, double uy, double uz, double *feq)
{
    const double u[3] = {ux, uy, uz};
    const double usq = (ux * ux + uy * uy) + uz * uz;
    for (int i = 0; i < Q; i++) {
        const double cu = c_dot_u(i, u);
        const double t = ((1.0 + 3.0 * cu) + 4.5 * (cu * cu)) - 1.5 * usq;
        feq[i] = (weight(i) * rho) * t;
    }
}

/* Collision of one cell's gathered populations g into out. */
static void collide(const double g[Q], double omega, double out[Q])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++)
        rho = rho + g[i];
    for (int a = 0; a < 3; a++)
        for (int i = 0; i < Q; i++) {
            if (CV[i][a] == 1)
                j[a] = j[a] + g[i];
            else if (CV[i][a] == -1)
                j[a] = j[a] - g[i];
        }
    double feq[Q];
    oracle_lbm_equilibrium(rho, j[0] / rho, j[1] / rho, j[2] / rho, feq);
    for (int i = 0; i < Q; i++)
        out[i] = g[i] - omega * (g[i] - feq[i]);
}

static long wrap(long v, long n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* One time step (streaming, then collision) from f into out. */
static void lbm_step(long nx, long ny, long nz, const double *f, double *out, double omega)
{
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double g[Q], o[Q];
                for (int i = 0; i < Q; i++) {
                    const long xs = wrap(x - CV[i][0], nx), ys = wrap(y - CV[i][1], ny);
                    const long zs = wrap(z - CV[i][2], nz);
                    g[i] = f[(size_t)i * n + (size_t)xs + (size_t)nx * ((size_t)ys + (size_t)ny * (size_t)zs)];
                }
                collide(g, omega, o);
                const size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z);
                for (int i = 0; i < Q; i++)
                    out[(size_t)i * n + c] = o[i];
            }
}

/*
 * T time steps from the populations f0 (19 * nx*ny*nz values); out receives
 * the populations after step T (out may equal f0; T = 0 copies).  Returns 0,
 * or -1 on bad arguments or allocation failure.
 */
int oracle_lbm_d3q19(long nx, long ny, long nz, const double *f0, double *out, double omega, int T,
                     int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || !f0 || !out)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const size_t total = (size_t)Q * (size_t)nx * (size_t)ny * (size_t)nz;
    double *a = malloc(total * sizeof(double)), *b = malloc(total * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, f0, total * sizeof(double));
    for (int s = 0; s < T; s++) {
        lbm_step(nx, ny, nz, a, b, omega);
        double *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, total * sizeof(double));
    free(a);
    free(b);
    return 0;
}
