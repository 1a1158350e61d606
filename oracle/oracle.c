/*
 * CPU oracle for the 3D Jacobi hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg load this library.  The product path never calls it and shares no code
 * with it.  Every routine is the plain definition, written for a reader who
 * checks it against the paper by eye: no blocking, no fusion, no reordering.
 *
 * Arithmetic: IEEE binary64, round to nearest even.  Built with
 * -O2 -ffp-contract=off and without -ffast-math, so every + and / below is one
 * correctly rounded operation, in the order written.
 *
 * Grid layout (all routines): a dense array of (nx+2)*(ny+2)*(nz+2) doubles,
 * element (i,j,k) at  i + (nx+2)*j + (nx+2)*(ny+2)*k,  0 <= i <= nx+1 etc.
 * Index 0 and n+1 on any axis is the fixed Dirichlet shell; 1..n is the
 * interior.  Only the six face layers of the shell are ever read (a cell on a
 * shell edge or corner has no interior neighbour).
 *
 * Readings taken where the paper is silent (each one is also listed with the
 * design notes of the project):
 *   - the six neighbours are summed left to right in the order the Jacobi
 *     update is printed (i-1, i+1, j-1, j+1, k-1, k+1), then the sum is divided
 *     by 6 with one correctly rounded division;
 *   - the shell never changes: both grids of the ping-pong pair carry it;
 *   - sweep s reads the grid written by sweep s-1 ("A and B in turn").
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, k) ((size_t)(i) + sy * (size_t)(j) + sz * (size_t)(k))

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_max_threads(int nthreads)
{
#ifdef _OPENMP
    set_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/*
 * One Jacobi sweep (the update equation of Sect. 1.1): for every interior cell,
 *   B(i,j,k) = ( A(i-1,j,k) + A(i+1,j,k) + A(i,j-1,k) + A(i,j+1,k)
 *              + A(i,j,k-1) + A(i,j,k+1) ) / 6,
 * summed left to right.  When rhs is non-NULL its value at the cell is added
 * as a seventh term before the division: the Jacobi step for the system
 * (6I - adjacency) e = rhs with a zero shell.  The shell of B is not touched.
 */
static void sweep(long nx, long ny, long nz, const double *A, double *B,
                  const double *rhs)
{
    const size_t sy = (size_t)nx + 2, sz = sy * ((size_t)ny + 2);
#pragma omp parallel for schedule(static)
    for (long k = 1; k <= nz; k++)
        for (long j = 1; j <= ny; j++)
            for (long i = 1; i <= nx; i++) {
                double s = A[IDX(i - 1, j, k)];
                s = s + A[IDX(i + 1, j, k)];
                s = s + A[IDX(i, j - 1, k)];
                s = s + A[IDX(i, j + 1, k)];
                s = s + A[IDX(i, j, k - 1)];
                s = s + A[IDX(i, j, k + 1)];
                if (rhs)
                    s = s + rhs[IDX(i, j, k)];
                B[IDX(i, j, k)] = s / 6.0;
            }
}

static size_t ncells(long nx, long ny, long nz)
{
    return ((size_t)nx + 2) * ((size_t)ny + 2) * ((size_t)nz + 2);
}

/*
 * T successive sweeps, grids A and B written in turn.  u holds level 0
 * (interior and shell); out receives level T (same layout).  u and out may be
 * the same array.  T = 0 copies u.  Returns 0, or -1 on bad arguments or
 * allocation failure.
 */
int oracle_sweeps(long nx, long ny, long nz, const double *u, double *out,
                  int T, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || !u || !out)
        return -1;
    set_threads(nthreads);
    const size_t n = ncells(nx, ny, nz);
    double *a = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, u, n * sizeof(double));
    memcpy(b, u, n * sizeof(double)); /* B carries the same shell */
    for (int s = 1; s <= T; s++) {
        sweep(nx, ny, nz, a, b, NULL);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(out, a, n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/*
 * Level T at the single cell (pi,pj,pk), computed from its domain of
 * dependence only.  Level T at a cell depends on level 0 within L-infinity
 * distance T, so the routine copies that box of u (clipped to the array) and
 * runs the same sweeps as oracle_sweeps on a box that shrinks by one cell per
 * side and sweep.  Every value it computes is the value oracle_sweeps computes
 * for the same cell and level, so the result is bitwise identical.
 * Returns NaN on bad arguments.
 */
double oracle_point(long nx, long ny, long nz, const double *u, int T,
                    long pi, long pj, long pk)
{
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || !u || pi < 0 || pj < 0 ||
        pk < 0 || pi > nx + 1 || pj > ny + 1 || pk > nz + 1)
        return NAN;
    const size_t sy = (size_t)nx + 2, sz = sy * ((size_t)ny + 2);
    if (T == 0 || pi == 0 || pj == 0 || pk == 0 || pi == nx + 1 ||
        pj == ny + 1 || pk == nz + 1)
        return u[IDX(pi, pj, pk)];
    /* box of level-0 values: [lo, hi] per axis, inside the array */
    long lo[3], hi[3], p[3] = {pi, pj, pk}, n[3] = {nx, ny, nz};
    for (int d = 0; d < 3; d++) {
        lo[d] = p[d] - T < 0 ? 0 : p[d] - T;
        hi[d] = p[d] + T > n[d] + 1 ? n[d] + 1 : p[d] + T;
    }
    const long bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1,
               bz = hi[2] - lo[2] + 1;
    const size_t bn = (size_t)bx * by * bz;
    double *a = malloc(bn * sizeof(double)), *b = malloc(bn * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return NAN;
    }
#define BIDX(i, j, k) \
    ((size_t)((i) - lo[0]) + (size_t)bx * ((size_t)((j) - lo[1]) + (size_t)by * (size_t)((k) - lo[2])))
    for (long k = lo[2]; k <= hi[2]; k++)
        for (long j = lo[1]; j <= hi[1]; j++)
            for (long i = lo[0]; i <= hi[0]; i++)
                a[BIDX(i, j, k)] = b[BIDX(i, j, k)] = u[IDX(i, j, k)];
    for (int s = 1; s <= T; s++) {
        const long r = T - s; /* cells within distance r of p are needed */
        long ulo[3], uhi[3];
        for (int d = 0; d < 3; d++) {
            ulo[d] = p[d] - r < 1 ? 1 : p[d] - r;
            uhi[d] = p[d] + r > n[d] ? n[d] : p[d] + r;
        }
        for (long k = ulo[2]; k <= uhi[2]; k++)
            for (long j = ulo[1]; j <= uhi[1]; j++)
                for (long i = ulo[0]; i <= uhi[0]; i++) {
                    double s6 = a[BIDX(i - 1, j, k)];
                    s6 = s6 + a[BIDX(i + 1, j, k)];
                    s6 = s6 + a[BIDX(i, j - 1, k)];
                    s6 = s6 + a[BIDX(i, j + 1, k)];
                    s6 = s6 + a[BIDX(i, j, k - 1)];
                    s6 = s6 + a[BIDX(i, j, k + 1)];
                    b[BIDX(i, j, k)] = s6 / 6.0;
                }
        double *tmp = a;
        a = b;
        b = tmp;
    }
    const double v = a[BIDX(pi, pj, pk)];
#undef BIDX
    free(a);
    free(b);
    return v;
}

/*
 * T sweeps of the right-hand-side form: e0 = 0 everywhere (zero shell), then
 *   e_s(i,j,k) = ( sum of the six neighbours of e_{s-1}, left to right,
 *                  + rhs(i,j,k) ) / 6.
 * This is Jacobi's method for (6I - adjacency) e = rhs on the interior.
 * rhs and e_out use the grid layout; the shell of rhs is ignored and the
 * shell of e_out is written as zero.
 */
int oracle_rhs_sweeps(long nx, long ny, long nz, const double *rhs,
                      double *e_out, int T, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || !rhs || !e_out)
        return -1;
    set_threads(nthreads);
    const size_t n = ncells(nx, ny, nz);
    double *a = calloc(n, sizeof(double)), *b = calloc(n, sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    for (int s = 1; s <= T; s++) {
        sweep(nx, ny, nz, a, b, rhs);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(e_out, a, n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/*
 * Residual of the Laplace system whose fixed point is the Jacobi iteration:
 * with the shell of x as the Dirichlet data g,
 *   r(i,j,k) = (sum of the six neighbours of x, left to right) - 6*x(i,j,k),
 * i.e. b - A x with A = 6I - (interior adjacency) and b = sum of the shell
 * neighbours.  6*x is rounded before the subtraction.  The shell of r is
 * written as zero.  Returns the squared 2-norm over the interior, summed in
 * storage order (k outer, i inner), or NaN on bad arguments.
 */
double oracle_residual(long nx, long ny, long nz, const double *x, double *r)
{
    if (nx < 1 || ny < 1 || nz < 1 || !x || !r)
        return NAN;
    const size_t sy = (size_t)nx + 2, sz = sy * ((size_t)ny + 2);
    memset(r, 0, ncells(nx, ny, nz) * sizeof(double));
    double norm2 = 0.0;
    for (long k = 1; k <= nz; k++)
        for (long j = 1; j <= ny; j++)
            for (long i = 1; i <= nx; i++) {
                double s = x[IDX(i - 1, j, k)];
                s = s + x[IDX(i + 1, j, k)];
                s = s + x[IDX(i, j - 1, k)];
                s = s + x[IDX(i, j + 1, k)];
                s = s + x[IDX(i, j, k - 1)];
                s = s + x[IDX(i, j, k + 1)];
                const double six_x = 6.0 * x[IDX(i, j, k)];
                const double v = s - six_x;
                r[IDX(i, j, k)] = v;
                norm2 = norm2 + v * v;
            }
    return norm2;
}

/*
 * Adjoint of T sweeps.  The forward map is linear: with u0 the interior and g
 * the shell, level s is  x_s = M x_{s-1} + G g,  M = (interior adjacency)/6,
 * and the output shell equals g.  Given grad_out = dL/d(level T) on the whole
 * array, the gradient with respect to the input array is
 *   interior:        lambda_0, where lambda_T = interior of grad_out and
 *                    lambda_{s-1} = M lambda_s (a sweep with a zero shell);
 *   face-shell cell: grad_out(b) + S_b / 6, where
 *                    S_b = lambda_T(in(b)) + lambda_{T-1}(in(b)) + ... + lambda_1(in(b))
 *                    summed in that order, in(b) the interior cell next to b;
 *   edge / corner:   grad_out(b) (no interior neighbour reads it).
 * grad_in may alias grad_out.
 */
int oracle_adjoint(long nx, long ny, long nz, const double *grad_out,
                   double *grad_in, int T, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || !grad_out || !grad_in)
        return -1;
    set_threads(nthreads);
    const size_t sy = (size_t)nx + 2, sz = sy * ((size_t)ny + 2);
    const size_t n = ncells(nx, ny, nz);
    double *a = calloc(n, sizeof(double)), *b = calloc(n, sizeof(double));
    double *S = calloc(n, sizeof(double));
    if (!a || !b || !S) {
        free(a);
        free(b);
        free(S);
        return -1;
    }
    for (long k = 1; k <= nz; k++)
        for (long j = 1; j <= ny; j++)
            for (long i = 1; i <= nx; i++)
                a[IDX(i, j, k)] = grad_out[IDX(i, j, k)];
    for (int s = T; s >= 1; s--) {
        /* a holds lambda_s: add it to the running sum of each face-shell cell */
        for (long k = 1; k <= nz; k++)
            for (long j = 1; j <= ny; j++) {
                S[IDX(0, j, k)] = S[IDX(0, j, k)] + a[IDX(1, j, k)];
                S[IDX(nx + 1, j, k)] = S[IDX(nx + 1, j, k)] + a[IDX(nx, j, k)];
            }
        for (long k = 1; k <= nz; k++)
            for (long i = 1; i <= nx; i++) {
                S[IDX(i, 0, k)] = S[IDX(i, 0, k)] + a[IDX(i, 1, k)];
                S[IDX(i, ny + 1, k)] = S[IDX(i, ny + 1, k)] + a[IDX(i, ny, k)];
            }
        for (long j = 1; j <= ny; j++)
            for (long i = 1; i <= nx; i++) {
                S[IDX(i, j, 0)] = S[IDX(i, j, 0)] + a[IDX(i, j, 1)];
                S[IDX(i, j, nz + 1)] = S[IDX(i, j, nz + 1)] + a[IDX(i, j, nz)];
            }
        sweep(nx, ny, nz, a, b, NULL); /* shells of a and b stay zero */
        double *tmp = a;
        a = b;
        b = tmp;
    }
    for (long k = 0; k <= nz + 1; k++)
        for (long j = 0; j <= ny + 1; j++)
            for (long i = 0; i <= nx + 1; i++) {
                const int on_i = (i == 0 || i == nx + 1);
                const int on_j = (j == 0 || j == ny + 1);
                const int on_k = (k == 0 || k == nz + 1);
                const int nshell = on_i + on_j + on_k;
                const size_t p = IDX(i, j, k);
                if (nshell == 0)
                    grad_in[p] = a[p];
                else if (nshell == 1)
                    grad_in[p] = grad_out[p] + S[p] / 6.0;
                else
                    grad_in[p] = grad_out[p];
            }
    free(a);
    free(b);
    free(S);
    return 0;
}

/*
 * All-FP64 Jacobi solve of the Laplace problem: starting from x (shell = g,
 * interior = initial guess), sweep with the update equation and, every
 * check_every sweeps, compute the residual norm; stop as soon as
 * ||r|| <= tol * ||r_initial||, or after max_sweeps sweeps.  x receives the
 * final iterate.  *sweeps_done and *rel_res report the sweep count and the
 * final ||r|| / ||r_initial||.  Returns 0 when converged, 1 when max_sweeps
 * was reached first, -1 on bad arguments.
 */
int oracle_jacobi_solve(long nx, long ny, long nz, double *x, double tol,
                        int check_every, long max_sweeps, int nthreads,
                        long *sweeps_done, double *rel_res)
{
    if (nx < 1 || ny < 1 || nz < 1 || !x || check_every < 1 || max_sweeps < 0 ||
        !(tol >= 0.0))
        return -1;
    set_threads(nthreads);
    const size_t n = ncells(nx, ny, nz);
    double *r = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
    if (!r || !b) {
        free(r);
        free(b);
        return -1;
    }
    memcpy(b, x, n * sizeof(double));
    const double r0 = sqrt(oracle_residual(nx, ny, nz, x, r));
    double rel = r0 > 0.0 ? 1.0 : 0.0;
    long done = 0;
    double *a = x, *c = b;
    while (rel > tol && done < max_sweeps) {
        sweep(nx, ny, nz, a, c, NULL);
        double *tmp = a;
        a = c;
        c = tmp;
        done++;
        if (done % check_every == 0 || done == max_sweeps)
            rel = sqrt(oracle_residual(nx, ny, nz, a, r)) / r0;
    }
    if (a != x)
        memcpy(x, a, n * sizeof(double));
    free(r);
    free(b);
    if (sweeps_done)
        *sweeps_done = done;
    if (rel_res)
        *rel_res = rel;
    return rel <= tol ? 0 : 1;
}

/*
 * The host's copy bandwidth M_s (bytes read plus bytes written per second) in
 * the manner of the STREAM COPY benchmark that Eq. 2 of the paper takes its
 * memory bandwidth from: b[i] = a[i] over n doubles on all threads (each
 * thread first touches the part it copies), the best of `reps` timed copies.
 * Not the method: the CPU baseline's reference figure P0 = M_s / 16 B.
 * Returns -1 on allocation failure.
 */
double oracle_copy_bandwidth(long n, int reps, int nthreads)
{
    if (n < 1 || reps < 1)
        return -1.0;
    set_threads(nthreads);
    double *a = malloc((size_t)n * sizeof(double)), *b = malloc((size_t)n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -1.0;
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        a[i] = 1.0;
        b[i] = 0.0;
    }
    double best = 0.0;
    for (int r = 0; r <= reps; r++) {
#ifdef _OPENMP
        const double t0 = omp_get_wtime();
#endif
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++)
            b[i] = a[i];
#ifdef _OPENMP
        const double dt = omp_get_wtime() - t0;
#else
        const double dt = 1.0;
#endif
        if (r > 0 && dt > 0.0) {      /* the first copy is a warm-up */
            const double bw = 2.0 * (double)n * sizeof(double) / dt;
            if (bw > best)
                best = bw;
        }
    }
    volatile double sink = b[n / 2];
    (void)sink;
    free(a);
    free(b);
    return best;
}
