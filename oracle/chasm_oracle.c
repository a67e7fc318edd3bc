/*
 * chasm_oracle.c -- FP64 CPU oracle for the characteristic (spatial-advection)
 * step of the CHASM scheme: Xiong, Zhang, Shao, "A characteristic-spectral-mixed
 * scheme for six-dimensional Wigner-Coulomb dynamics" (arXiv:2205.02380).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the HIP library; the two meet only through the
 * seeded input generator.
 *
 * Everything is FP64 and deliberately plain: dense Gauss-Jordan / Gaussian
 * elimination with partial pivoting, the B-spline evaluated from its piecewise
 * definition, and one output array per sweep.  No blocking, fusion or reordering.
 *
 * One axis, in the notation used throughout:
 *   nodes   x_i = x_lo + i*h, i = 0..N-1  (the paper's x_0..x_N with its N = our N-1)
 *   patches of M cells, p = ceil((N-1)/M); patch l spans nodes
 *           s_l = l*M .. e_l = min((l+1)*M, N-1), m_l = e_l - s_l cells;
 *           neighbouring patches share their end node (Sec. 3.1, eq. 3.1)
 *   interfaces I_q = q*M for q < p, I_p = N-1 (the node where patch q-1 meets q,
 *           plus both line ends)
 *   shift   f_new(x_j) = s(x_j - alpha*h), alpha = k*dt/h with hbar = m = 1
 *           (characteristic flow A_tau, Sec. 2.2, eq. 2.6)
 *
 * Readings of the paper that this file commits to (each is also listed in the
 * design notes):
 *   - interface derivatives at every interface use rows of the inverse of the
 *     natural-BC global matrix (eq. 3.5's A-tilde), truncated to |j - I| <= g
 *     (g = n_nb, eqs. 3.3-3.5);
 *   - the ghost splines beyond the outer line ends carry coefficient 0 (Sec. 3.1.3);
 *   - the patch whose cells contain the departure point evaluates it (the upwind
 *     patch of the correction procedure, Sec. 3.1.3);
 *   - shifts of any size: the departure cell is floor(j - alpha);
 *   - optional closure NEUMANN: the global matrix takes the Hermite boundary rows of
 *     eq. 2.13 with zero end slopes (the Neumann condition the paper names as the
 *     alternative to the natural one); stencils are rows of its inverse;
 *   - optional closure HERMITE: the same matrix with given end slopes phi_L, phi_R
 *     (eq. 2.13) on the right-hand side of its boundary rows.  The interface slope
 *     then has a data part (truncated to |j - I| <= g as above) and the parts
 *     c_L(I) phi_L + c_R(I) phi_R from the inverse's columns of the boundary rows;
 *     those two columns belong to the virtual nodes -1 and N one cell beyond the
 *     ends and are kept under the same distance rule: |(-1) - I| <= g, |N - I| <= g;
 *   - optional closure POLY3 (not in the paper): the truncated stencil rows get the
 *     minimum-norm correction that makes them exact for cubic data, and the outer
 *     ghost coefficient is extrapolated by a zero fourth difference, so cubic
 *     polynomials are carried exactly.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CLOSURE_PMBC 0
#define ORACLE_CLOSURE_POLY3 1
#define ORACLE_CLOSURE_NEUMANN 2
#define ORACLE_CLOSURE_HERMITE 3

/* ------------------------------------------------------------------------- */
/* Cubic B-spline centred at 0, support [-2, 2]: eq. (2.10) with x = x_nu + t*h. */
double chasm_oracle_bspline(double t)
{
    double u;
    if (t <= -2.0 || t >= 2.0) return 0.0;
    if (t < -1.0) { /* x in [x_{nu-2}, x_{nu-1}] */
        u = t + 2.0;
        return u * u * u / 6.0;
    }
    if (t < 0.0) {  /* x in [x_{nu-1}, x_nu] */
        u = t + 1.0;
        return -u * u * u / 2.0 + u * u / 2.0 + u / 2.0 + 1.0 / 6.0;
    }
    if (t < 1.0) {  /* x in [x_nu, x_{nu+1}] */
        u = 1.0 - t;
        return -u * u * u / 2.0 + u * u / 2.0 + u / 2.0 + 1.0 / 6.0;
    }
    u = 2.0 - t;    /* x in [x_{nu+1}, x_{nu+2}] */
    return u * u * u / 6.0;
}

int chasm_oracle_npatch(int N, int M)
{
    if (N < 2 || M < 1) return -1;
    return (N - 1 + M - 1) / M;
}

/* ------------------------------------------------------------------------- */
/* Dense linear algebra (plain, partial pivoting). */

/* Solve a x = b in place (a: n x n row-major, destroyed; b overwritten by x). */
static int dense_solve(int n, double *a, double *b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(a[col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            double v = fabs(a[r * n + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                double t = a[col * n + c]; a[col * n + c] = a[piv * n + c]; a[piv * n + c] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = a[r * n + col] / a[col * n + col];
            if (f == 0.0) continue;
            for (int c = col; c < n; ++c) a[r * n + c] -= f * a[col * n + c];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= a[r * n + c] * b[c];
        b[r] = s / a[r * n + r];
    }
    return 0;
}

/* Gauss-Jordan inverse (a destroyed). */
static int gj_inverse(int n, double *a, double *inv)
{
    for (int i = 0; i < n * n; ++i) inv[i] = 0.0;
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(a[col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            double v = fabs(a[r * n + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                double t = a[col * n + c]; a[col * n + c] = a[piv * n + c]; a[piv * n + c] = t;
                t = inv[col * n + c]; inv[col * n + c] = inv[piv * n + c]; inv[piv * n + c] = t;
            }
        }
        double d = a[col * n + col];
        for (int c = 0; c < n; ++c) { a[col * n + c] /= d; inv[col * n + c] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = a[r * n + col];
            if (f == 0.0) continue;
            for (int c = 0; c < n; ++c) {
                a[r * n + c] -= f * a[col * n + c];
                inv[r * n + c] -= f * inv[col * n + c];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Inverse of the natural-BC global spline matrix A-tilde (Sec. 3.1.2, before
 * eq. 3.5).  Unknowns eta_{-1..N} sit at positions 0..N+1.  Rows:
 *   0      : s''(x_0) = 0      (eq. 2.14)
 *   1..N   : interpolation at node i = row-1 (eq. 2.12)
 *   N+1    : s''(x_{N-1}) = 0  (eq. 2.14)
 * inv is (N+2) x (N+2) row-major.  Returns 0 on success. */
int chasm_oracle_global_inverse(int N, double h, int bc, double *inv);

int chasm_oracle_natural_inverse(int N, double h, double *inv)
{
    return chasm_oracle_global_inverse(N, h, 0, inv);
}

/* The global spline matrix with either boundary rows: bc 0 natural (eq. 2.14),
 * bc 1 Neumann, i.e. the Hermite rows of eq. 2.13 with phi_L = phi_R = 0:
 *   row 0   : (eta_1 - eta_{-1}) / 2h = 0
 *   row N+1 : (eta_N - eta_{N-2}) / 2h = 0
 * (the right-hand sides of the boundary rows are 0, so only data columns matter). */
int chasm_oracle_global_inverse(int N, double h, int bc, double *inv)
{
    if (N < 2 || !(h > 0.0) || (bc != 0 && bc != 1)) return -1;
    int n = N + 2;
    double *a = (double *)calloc((size_t)n * n, sizeof(double));
    if (!a) return -2;
    double ih2 = 1.0 / (h * h), i2h = 1.0 / (2.0 * h);
    if (bc == 0) {
        a[0 * n + 0] = ih2; a[0 * n + 1] = -2.0 * ih2; a[0 * n + 2] = ih2;
    } else {
        a[0 * n + 0] = -i2h; a[0 * n + 2] = i2h;
    }
    for (int i = 0; i < N; ++i) {
        int r = i + 1;
        a[r * n + i] += 1.0 / 6.0;        /* eta_{i-1} */
        a[r * n + i + 1] += 2.0 / 3.0;    /* eta_i     */
        a[r * n + i + 2] += 1.0 / 6.0;    /* eta_{i+1} */
    }
    if (bc == 0) {
        a[(N + 1) * n + (N - 1)] = ih2; a[(N + 1) * n + N] = -2.0 * ih2; a[(N + 1) * n + (N + 1)] = ih2;
    } else {
        a[(N + 1) * n + (N - 1)] = -i2h; a[(N + 1) * n + (N + 1)] = i2h;
    }
    int rc = gj_inverse(n, a, inv);
    free(a);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Interface stencils (eqs. 3.4-3.5): d_I = sum_j c_j(I) phi_j approximates s'(x_I)
 * of the global natural spline, with c_j(I) = (b_{I+1,j} - b_{I-1,j}) / (2h) taken
 * from A-tilde^{-1} and kept for |j - I| <= g.  Output: (p+1) dense rows of length
 * N (zeros outside the band), row q for interface I_q.
 * closure POLY3 adds the minimum-2-norm correction so that each row differentiates
 * cubic data exactly. */
int chasm_oracle_stencils_bc(int N, int M, int g, double h, int closure, double phi_l, double phi_r,
                             double *c, double *bias);

int chasm_oracle_stencils(int N, int M, int g, double h, int closure, double *c)
{
    if (closure == ORACLE_CLOSURE_HERMITE) return -1;
    return chasm_oracle_stencils_bc(N, M, g, h, closure, 0.0, 0.0, c, NULL);
}

/* The rows above and, for closure HERMITE, bias[q] = c_L(I_q) phi_L + c_R(I_q) phi_R
 * (truncated; bias may be NULL for the other closures, else it is set to 0). */
int chasm_oracle_stencils_bc(int N, int M, int g, double h, int closure, double phi_l, double phi_r,
                             double *c, double *bias)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1 || g < 1 || !(h > 0.0)) return -1;
    if (closure != ORACLE_CLOSURE_PMBC && closure != ORACLE_CLOSURE_POLY3 && closure != ORACLE_CLOSURE_NEUMANN &&
        closure != ORACLE_CLOSURE_HERMITE)
        return -1;
    if (closure == ORACLE_CLOSURE_HERMITE && !bias) return -1;
    int n = N + 2;
    double *inv = (double *)malloc((size_t)n * n * sizeof(double));
    if (!inv) return -2;
    int hermite_rows = closure == ORACLE_CLOSURE_NEUMANN || closure == ORACLE_CLOSURE_HERMITE;
    int rc = chasm_oracle_global_inverse(N, h, hermite_rows ? 1 : 0, inv);
    if (rc) { free(inv); return rc; }
    memset(c, 0, (size_t)(p + 1) * N * sizeof(double));
    if (bias) memset(bias, 0, (size_t)(p + 1) * sizeof(double));
    for (int q = 0; q <= p; ++q) {
        int I = (q < p) ? q * M : N - 1;
        double *row = c + (size_t)q * N;
        if (closure == ORACLE_CLOSURE_HERMITE) {
            /* boundary-row columns: phi_L is the right-hand side of row 0, phi_R of row N+1 */
            if (abs(-1 - I) <= g) bias[q] += (inv[(size_t)(I + 2) * n + 0] - inv[(size_t)I * n + 0]) / (2.0 * h) * phi_l;
            if (abs(N - I) <= g)
                bias[q] += (inv[(size_t)(I + 2) * n + (N + 1)] - inv[(size_t)I * n + (N + 1)]) / (2.0 * h) * phi_r;
        }
        for (int j = 0; j < N; ++j) {
            if (abs(j - I) > g) continue;
            /* eta_{I+1} at position I+2, eta_{I-1} at position I; data phi_j is column j+1 */
            row[j] = (inv[(size_t)(I + 2) * n + (j + 1)] - inv[(size_t)I * n + (j + 1)]) / (2.0 * h);
        }
        if (closure == ORACLE_CLOSURE_POLY3) {
            /* Moment conditions sum_j row[j] * (j-I)^q = delta_{q1} / h, q = 0..3.
             * Correction row += V lambda with (V^T V) lambda = e - V^T row. */
            int lo = I - g < 0 ? 0 : I - g, hi = I + g > N - 1 ? N - 1 : I + g;
            if (hi - lo + 1 < 4) { free(inv); return -1; }
            double G[16], r[4];
            for (int a = 0; a < 4; ++a) {
                r[a] = (a == 1) ? 1.0 / h : 0.0;
                for (int b = 0; b < 4; ++b) G[a * 4 + b] = 0.0;
            }
            for (int j = lo; j <= hi; ++j) {
                double t = (double)(j - I), pw[4] = {1.0, t, t * t, t * t * t};
                for (int a = 0; a < 4; ++a) {
                    r[a] -= pw[a] * row[j];
                    for (int b = 0; b < 4; ++b) G[a * 4 + b] += pw[a] * pw[b];
                }
            }
            if (dense_solve(4, G, r)) { free(inv); return -3; }
            for (int j = lo; j <= hi; ++j) {
                double t = (double)(j - I), pw[4] = {1.0, t, t * t, t * t * t};
                for (int a = 0; a < 4; ++a) row[j] += pw[a] * r[a];
            }
        }
    }
    free(inv);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Patch coefficients for one line.  For patch l the unknowns eta_{-1..m+1} solve
 * the (m+3) x (m+3) system of Sec. 3.1.2 step (5): effective Hermite conditions
 * (eq. 2.13) at both patch ends with slopes d_{I_l}, d_{I_{l+1}}, and interpolation
 * (eq. 2.12) at the m+1 patch nodes.  Result: eta[l * (M+5) + (nu+2)] for
 * nu = -2..m_l+2, where nu = -2 and nu = m_l+2 are the ghost coefficients. */
static int patch_coefficients(int N, int M, double h, int closure, const double *c, const double *bias,
                              const double *phi, double *d, double *eta, double *work)
{
    int p = chasm_oracle_npatch(N, M);
    for (int q = 0; q <= p; ++q) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += c[(size_t)q * N + j] * phi[j];
        d[q] = s + (bias ? bias[q] : 0.0);
    }
    int stride = M + 5;
    for (int l = 0; l < p; ++l) {
        int s = l * M, e = (l + 1) * M < N - 1 ? (l + 1) * M : N - 1, m = e - s;
        int n = m + 3;
        double *a = work, *b = work + (size_t)n * n;
        memset(a, 0, (size_t)n * n * sizeof(double));
        /* row 0: (eta_1 - eta_{-1}) / (2h) = d_L ; position u = nu + 1 */
        a[0 * n + 0] = -1.0 / (2.0 * h);
        a[0 * n + 2] = 1.0 / (2.0 * h);
        b[0] = d[l];
        for (int i = 0; i <= m; ++i) {
            a[(i + 1) * n + i] = 1.0 / 6.0;
            a[(i + 1) * n + i + 1] = 2.0 / 3.0;
            a[(i + 1) * n + i + 2] = 1.0 / 6.0;
            b[i + 1] = phi[s + i];
        }
        /* last row: (eta_{m+1} - eta_{m-1}) / (2h) = d_R */
        a[(m + 2) * n + m] = -1.0 / (2.0 * h);
        a[(m + 2) * n + m + 2] = 1.0 / (2.0 * h);
        b[m + 2] = d[l + 1];
        if (dense_solve(n, a, b)) return -3;
        double *el = eta + (size_t)l * stride;
        for (int k = 0; k < stride; ++k) el[k] = 0.0;
        for (int u = 0; u < n; ++u) el[u + 1] = b[u];   /* nu = u - 1 -> slot nu + 2 */
        if (closure == ORACLE_CLOSURE_POLY3) {
            /* zero fourth difference beyond the outer line ends */
            if (l == 0)
                el[0] = 4.0 * el[1] - 6.0 * el[2] + 4.0 * el[3] - el[4];
            if (l == p - 1)
                el[m + 4] = 4.0 * el[m + 3] - 6.0 * el[m + 2] + 4.0 * el[m + 1] - el[m];
        }
    }
    return 0;
}

/* Evaluate the shifted patched spline: for each output node j the departure point
 * is t = j - alpha (units of h from x_0), its cell floor(t); the patch owning that
 * cell (clamped to the outer patches) sums its coefficients against B directly. */
static void patch_evaluate(int N, int M, double alpha, const double *eta, double *out)
{
    int p = chasm_oracle_npatch(N, M);
    int stride = M + 5;
    for (int j = 0; j < N; ++j) {
        double t = (double)j - alpha;
        double cell = floor(t);
        int l = (int)floor(cell / (double)M);
        if (l < 0) l = 0;
        if (l > p - 1) l = p - 1;
        int s = l * M, e = (l + 1) * M < N - 1 ? (l + 1) * M : N - 1, m = e - s;
        const double *el = eta + (size_t)l * stride;
        double y = t - (double)s, acc = 0.0;
        for (int nu = -2; nu <= m + 2; ++nu) acc += el[nu + 2] * chasm_oracle_bspline(y - (double)nu);
        out[j] = acc;
    }
}

/* Interface derivatives of one line: d[q] = sum_j c[q][j] phi[j], q = 0..p. */
int chasm_oracle_interface_derivs(int N, int M, const double *c, const double *phi, double *d)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1) return -1;
    for (int q = 0; q <= p; ++q) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += c[(size_t)q * N + j] * phi[j];
        d[q] = s;
    }
    return 0;
}

/* Patch coefficients of one line, exported for tests: eta is p x (M+5). */
int chasm_oracle_line_coefficients(int N, int M, double h, int closure, const double *c,
                                   const double *phi, double *eta)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1) return -1;
    int n = M + 3;
    double *d = (double *)malloc((size_t)(p + 1) * sizeof(double));
    double *work = (double *)malloc((size_t)(n * n + n) * sizeof(double));
    if (!d || !work) { free(d); free(work); return -2; }
    int rc = patch_coefficients(N, M, h, closure, c, NULL, phi, d, eta, work);
    free(d); free(work);
    return rc;
}

/* The same with the end-slope part of closure HERMITE (bias from chasm_oracle_stencils_bc). */
int chasm_oracle_line_coefficients_bc(int N, int M, double h, int closure, const double *c, const double *bias,
                                      const double *phi, double *eta)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1) return -1;
    int n = M + 3;
    double *d = (double *)malloc((size_t)(p + 1) * sizeof(double));
    double *work = (double *)malloc((size_t)(n * n + n) * sizeof(double));
    if (!d || !work) { free(d); free(work); return -2; }
    int rc = patch_coefficients(N, M, h, closure, c, bias, phi, d, eta, work);
    free(d); free(work);
    return rc;
}

/* One sweep of one line under closure HERMITE (or any closure, bias NULL). */
int chasm_oracle_line_bc(int N, int M, double h, int closure, const double *c, const double *bias, double alpha,
                         const double *phi, double *out)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1) return -1;
    double *eta = (double *)malloc((size_t)p * (M + 5) * sizeof(double));
    if (!eta) return -2;
    int rc = chasm_oracle_line_coefficients_bc(N, M, h, closure, c, bias, phi, eta);
    if (!rc) patch_evaluate(N, M, alpha, eta, out);
    free(eta);
    return rc;
}

/* One sweep of one line with precomputed stencils c ((p+1) x N). */
int chasm_oracle_line(int N, int M, double h, int closure, const double *c, double alpha,
                      const double *phi, double *out)
{
    int p = chasm_oracle_npatch(N, M);
    if (p < 1) return -1;
    double *eta = (double *)malloc((size_t)p * (M + 5) * sizeof(double));
    if (!eta) return -2;
    int rc = chasm_oracle_line_coefficients(N, M, h, closure, c, phi, eta);
    if (!rc) patch_evaluate(N, M, alpha, eta, out);
    free(eta);
    return rc;
}

/* Brute-force global reference: the natural spline of the whole line (eq. 2.15 with
 * eq. 2.14), no patches, ghosts eta_{-2} = eta_{N+1} = 0. */
int chasm_oracle_global_line_bc(int N, double h, int bc, double alpha, const double *phi, double *out);

int chasm_oracle_global_line(int N, double h, double alpha, const double *phi, double *out)
{
    return chasm_oracle_global_line_bc(N, h, 0, alpha, phi, out);
}

/* The same with the boundary rows of chasm_oracle_global_inverse (bc 0 natural,
 * bc 1 Neumann). */
int chasm_oracle_global_line_bc(int N, double h, int bc, double alpha, const double *phi, double *out)
{
    int n = N + 2;
    double *inv = (double *)malloc((size_t)n * n * sizeof(double));
    double *eta = (double *)malloc((size_t)n * sizeof(double));
    if (!inv || !eta) { free(inv); free(eta); return -2; }
    int rc = chasm_oracle_global_inverse(N, h, bc, inv);
    if (rc) { free(inv); free(eta); return rc; }
    for (int u = 0; u < n; ++u) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += inv[(size_t)u * n + (j + 1)] * phi[j];
        eta[u] = s;   /* eta_{u-1} */
    }
    for (int j = 0; j < N; ++j) {
        double t = (double)j - alpha, acc = 0.0;
        for (int nu = -1; nu <= N; ++nu) acc += eta[nu + 1] * chasm_oracle_bspline(t - (double)nu);
        out[j] = acc;
    }
    free(inv); free(eta);
    return 0;
}

/* Brute-force global reference of the Hermite condition with given end slopes:
 * eta = A^{-1} (phi_L, phi_0..phi_{N-1}, phi_R), no patches, ghosts 0. */
int chasm_oracle_global_line_hermite(int N, double h, double phi_l, double phi_r, double alpha, const double *phi,
                                     double *out)
{
    int n = N + 2;
    double *inv = (double *)malloc((size_t)n * n * sizeof(double));
    double *eta = (double *)malloc((size_t)n * sizeof(double));
    if (!inv || !eta) { free(inv); free(eta); return -2; }
    int rc = chasm_oracle_global_inverse(N, h, 1, inv);
    if (rc) { free(inv); free(eta); return rc; }
    for (int u = 0; u < n; ++u) {
        double s = inv[(size_t)u * n + 0] * phi_l + inv[(size_t)u * n + (N + 1)] * phi_r;
        for (int j = 0; j < N; ++j) s += inv[(size_t)u * n + (j + 1)] * phi[j];
        eta[u] = s;
    }
    for (int j = 0; j < N; ++j) {
        double t = (double)j - alpha, acc = 0.0;
        for (int nu = -1; nu <= N; ++nu) acc += eta[nu + 1] * chasm_oracle_bspline(t - (double)nu);
        out[j] = acc;
    }
    free(inv); free(eta);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 6-D step (Sec. 3.2): for each k-point independently, sweep x1 with
 * alpha_1 = k1*dt/h1, then x2, then x3, nsteps times.
 * cubes: nkp cubes of nx[2]*nx[1]*nx[0] values, x1 fastest.  If kidx is NULL the
 * cubes are all k-points in [k3][k2][k1] order (nkp = nk1*nk2*nk3); otherwise
 * kidx[3*i..3*i+2] = (i1, i2, i3) gives the k-point of cube i.
 * g: stencil half-width; M[d]: patch cells per axis.  nthreads <= 0: default. */
int chasm_oracle_advect6d_bc(const int nx[3], const double hx[3], const int nk[3],
                             const double klo[3], const double hk[3], const int M[3], int g,
                             int closure, const double slope_lo[3], const double slope_hi[3], double dt,
                             int nsteps, int nkp, const int *kidx, double *cubes, int nthreads);

int chasm_oracle_advect6d(const int nx[3], const double hx[3], const int nk[3],
                          const double klo[3], const double hk[3], const int M[3], int g,
                          int closure, double dt, int nsteps, int nkp, const int *kidx,
                          double *cubes, int nthreads)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    return chasm_oracle_advect6d_bc(nx, hx, nk, klo, hk, M, g, closure, zero, zero, dt, nsteps, nkp, kidx, cubes,
                                    nthreads);
}

/* The same with the end slopes of closure HERMITE per axis (ignored otherwise). */
int chasm_oracle_advect6d_bc(const int nx[3], const double hx[3], const int nk[3],
                             const double klo[3], const double hk[3], const int M[3], int g,
                             int closure, const double slope_lo[3], const double slope_hi[3], double dt,
                             int nsteps, int nkp, const int *kidx, double *cubes, int nthreads)
{
    if (nsteps < 0 || nkp < 0) return -1;
    if (!kidx && nkp != nk[0] * nk[1] * nk[2]) return -1;
    double *c[3] = {0, 0, 0}, *bias[3] = {0, 0, 0};
    int rc = 0;
    for (int d = 0; d < 3; ++d) {
        int p = chasm_oracle_npatch(nx[d], M[d]);
        if (p < 1) { rc = -1; break; }
        c[d] = (double *)malloc((size_t)(p + 1) * nx[d] * sizeof(double));
        bias[d] = (double *)malloc((size_t)(p + 1) * sizeof(double));
        if (!c[d] || !bias[d]) { rc = -2; break; }
        rc = chasm_oracle_stencils_bc(nx[d], M[d], g, hx[d], closure, slope_lo[d], slope_hi[d], c[d], bias[d]);
        if (rc) break;
    }
    if (rc) { for (int d = 0; d < 3; ++d) { free(c[d]); free(bias[d]); } return rc; }
    size_t cube = (size_t)nx[0] * nx[1] * nx[2];
    int nmax = nx[0] > nx[1] ? nx[0] : nx[1];
    if (nx[2] > nmax) nmax = nx[2];
    int mmax = M[0] > M[1] ? M[0] : M[1];
    if (M[2] > mmax) mmax = M[2];
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : err)
#endif
    {
        double *tmp = (double *)malloc(cube * sizeof(double));
        double *phi = (double *)malloc((size_t)nmax * sizeof(double));
        double *out = (double *)malloc((size_t)nmax * sizeof(double));
        double *eta = (double *)malloc((size_t)(nmax + 1) * (mmax + 5) * sizeof(double));
        double *dd = (double *)malloc((size_t)(nmax + 2) * sizeof(double));
        double *work = (double *)malloc((size_t)((mmax + 3) * (mmax + 3) + mmax + 3) * sizeof(double));
        if (!tmp || !phi || !out || !eta || !dd || !work) err = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int ip = 0; ip < nkp; ++ip) {
            if (err) continue;
            int ik[3];
            if (kidx) { ik[0] = kidx[3 * ip]; ik[1] = kidx[3 * ip + 1]; ik[2] = kidx[3 * ip + 2]; }
            else { ik[0] = ip % nk[0]; ik[1] = (ip / nk[0]) % nk[1]; ik[2] = ip / (nk[0] * nk[1]); }
            double *f = cubes + (size_t)ip * cube;
            for (int st = 0; st < nsteps && !err; ++st) {
                for (int d = 0; d < 3 && !err; ++d) {
                    double k = klo[d] + ik[d] * hk[d];
                    double alpha = k * dt / hx[d];
                    size_t stride = d == 0 ? 1 : (d == 1 ? (size_t)nx[0] : (size_t)nx[0] * nx[1]);
                    /* every line along axis d: the two other indices run over their ranges */
                    int oa = d == 0 ? 1 : 0, ob = d == 2 ? 1 : 2;
                    size_t sa = oa == 0 ? 1 : (size_t)nx[0], sb = ob == 1 ? (size_t)nx[0] : (size_t)nx[0] * nx[1];
                    for (int b = 0; b < nx[ob]; ++b)
                        for (int a = 0; a < nx[oa]; ++a) {
                            size_t base = (size_t)a * sa + (size_t)b * sb;
                            for (int i = 0; i < nx[d]; ++i) phi[i] = f[base + (size_t)i * stride];
                            if (patch_coefficients(nx[d], M[d], hx[d], closure, c[d], bias[d], phi, dd, eta, work)) {
                                err = 1;
                                break;
                            }
                            patch_evaluate(nx[d], M[d], alpha, eta, out);
                            for (int i = 0; i < nx[d]; ++i) tmp[base + (size_t)i * stride] = out[i];
                        }
                    memcpy(f, tmp, cube * sizeof(double));
                }
            }
        }
        free(tmp); free(phi); free(out); free(eta); free(dd); free(work);
    }
    for (int d = 0; d < 3; ++d) { free(c[d]); free(bias[d]); }
    return err ? -3 : 0;
}

/* ------------------------------------------------------------------------- */
/* FP64 pairwise sum of n terms term(i). */
typedef double (*term_fn)(const void *ctx, size_t i);

static double pairwise(const void *ctx, term_fn fn, size_t lo, size_t hi)
{
    if (hi - lo <= 64) {
        double s = 0.0;
        for (size_t i = lo; i < hi; ++i) s += fn(ctx, i);
        return s;
    }
    size_t mid = lo + (hi - lo) / 2;
    return pairwise(ctx, fn, lo, mid) + pairwise(ctx, fn, mid, hi);
}

typedef struct {
    const double *f;
    int nx[3], nk[3];
    double xlo[3], hx[3], klo[3], hk[3];
    int which;
} red_ctx;

static double red_term(const void *vctx, size_t i)
{
    const red_ctx *r = (const red_ctx *)vctx;
    double v = r->f[i];
    size_t t = i;
    int ix[3], ik[3];
    ix[0] = (int)(t % r->nx[0]); t /= r->nx[0];
    ix[1] = (int)(t % r->nx[1]); t /= r->nx[1];
    ix[2] = (int)(t % r->nx[2]); t /= r->nx[2];
    ik[0] = (int)(t % r->nk[0]); t /= r->nk[0];
    ik[1] = (int)(t % r->nk[1]); t /= r->nk[1];
    ik[2] = (int)t;
    switch (r->which) {
    case 0: return v;
    case 1: return v * v;
    case 2: case 3: case 4: { int d = r->which - 2; return (r->xlo[d] + ix[d] * r->hx[d]) * v; }
    default: { int d = r->which - 5; return (r->klo[d] + ik[d] * r->hk[d]) * v; }
    }
}

/* Diagnostics (Sec. 5, error metrics; integrals as grid sums): out[0] = V sum f,
 * out[1] = V sum f^2, out[2..4] = V sum x_d f, out[5..7] = V sum k_d f, with
 * V = prod h_d * prod hk_d.  f is the full field [nb][k3][k2][k1][x3][x2][x1]; the
 * batch index nb is summed over as well. */
int chasm_oracle_reduce(const int nx[3], const double xlo[3], const double hx[3], const int nk[3],
                        const double klo[3], const double hk[3], int nb, const double *f,
                        double out[8])
{
    red_ctx r;
    for (int d = 0; d < 3; ++d) {
        r.nx[d] = nx[d]; r.nk[d] = nk[d]; r.xlo[d] = xlo[d]; r.hx[d] = hx[d];
        r.klo[d] = klo[d]; r.hk[d] = hk[d];
    }
    size_t n1 = (size_t)nx[0] * nx[1] * nx[2] * nk[0] * nk[1] * nk[2];
    double V = hx[0] * hx[1] * hx[2] * hk[0] * hk[1] * hk[2];
    for (int w = 0; w < 8; ++w) {
        double s = 0.0;
        for (int b = 0; b < (nb < 1 ? 1 : nb); ++b) {
            r.f = f + (size_t)b * n1;
            r.which = w;
            s += pairwise(&r, red_term, 0, n1);
        }
        out[w] = V * s;
    }
    return 0;
}
