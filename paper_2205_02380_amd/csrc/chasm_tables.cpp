// chasm_tables.cpp -- FP64 table builder (host).  See chasm_tables.hpp.
#include "chasm_tables.hpp"

#include <cmath>
#include <cstdlib>

namespace chasm {

// The natural boundary condition s''(x_0) = 0 (eq. 2.14) together with the
// interpolation row at x_0 (eq. 2.12) gives eta_0 = phi_0 and eta_{-1} = 2 eta_0 - eta_1;
// likewise at the right end.  The remaining unknowns eta_1..eta_{N-2} solve
// eta_{i-1} + 4 eta_i + eta_{i+1} = 6 phi_i with eta_0, eta_{N-1} known: a symmetric,
// strictly diagonally dominant tridiagonal system, solved here column by column with
// the sweeping method for unit data.
bool natural_slope_rows(int N, double h, const std::vector<int>& ifaces, std::vector<double>& out)
{
    if (N < 2 || !(h > 0.0)) return false;
    const int n = N - 2;
    std::vector<double> cp(n > 0 ? n : 1), den(n > 0 ? n : 1);
    for (int i = 0; i < n; ++i) {
        den[i] = 4.0 - (i > 0 ? cp[i - 1] : 0.0);
        cp[i] = 1.0 / den[i];
    }
    std::vector<double> eta(N + 2), y(n > 0 ? n : 1);
    out.assign(ifaces.size() * (size_t)N, 0.0);
    for (int j = 0; j < N; ++j) {
        // eta[u] = eta_{u-1}
        const double e0 = (j == 0) ? 1.0 : 0.0, eN = (j == N - 1) ? 1.0 : 0.0;
        eta[1] = e0;
        eta[N] = eN;
        for (int i = 0; i < n; ++i) {                 // unknown eta_{i+1}
            double r = (j == i + 1) ? 6.0 : 0.0;
            if (i == 0) r -= e0;
            if (i == n - 1) r -= eN;
            y[i] = (r - (i > 0 ? y[i - 1] : 0.0)) / den[i];
        }
        for (int i = n - 1; i >= 0; --i) {
            if (i < n - 1) y[i] -= cp[i] * y[i + 1];
            eta[i + 2] = y[i];
        }
        eta[0] = 2.0 * eta[1] - eta[2];               // eta_{-1}
        eta[N + 1] = 2.0 * eta[N] - eta[N - 1];       // eta_N
        for (size_t q = 0; q < ifaces.size(); ++q) {
            const int I = ifaces[q];
            out[q * N + j] = (eta[I + 2] - eta[I]) / (2.0 * h);
        }
    }
    return true;
}

// The Neumann condition (eq. 2.13 with zero end slopes): eta_{-1} = eta_1 and eta_N =
// eta_{N-2}, so eta_0..eta_{N-1} solve [4 2; 1 4 1; ...; 2 4] eta = 6 phi, a strictly
// diagonally dominant tridiagonal system; the slopes at both ends are 0.
bool neumann_slope_rows(int N, double h, const std::vector<int>& ifaces, std::vector<double>& out)
{
    if (N < 2 || !(h > 0.0)) return false;
    std::vector<double> cp(N), den(N), y(N), eta(N + 2);
    for (int i = 0; i < N; ++i) {
        const double sub = i == N - 1 ? 2.0 : 1.0, sup = i == 0 ? 2.0 : 1.0;
        den[i] = 4.0 - (i > 0 ? sub * cp[i - 1] : 0.0);
        cp[i] = sup / den[i];
    }
    out.assign(ifaces.size() * (size_t)N, 0.0);
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < N; ++i) {
            const double sub = i == N - 1 ? 2.0 : 1.0;
            y[i] = ((i == j ? 6.0 : 0.0) - (i > 0 ? sub * y[i - 1] : 0.0)) / den[i];
        }
        for (int i = N - 2; i >= 0; --i) y[i] -= cp[i] * y[i + 1];
        for (int i = 0; i < N; ++i) eta[i + 1] = y[i];
        eta[0] = eta[2];
        eta[N + 1] = eta[N - 1];
        for (size_t q = 0; q < ifaces.size(); ++q) {
            const int I = ifaces[q];
            out[q * N + j] = (eta[I + 2] - eta[I]) / (2.0 * h);
        }
    }
    return true;
}

// The Hermite condition of eq. 2.13 with given end slopes phi_L, phi_R: eliminating
// eta_{-1} = eta_1 - 2h phi_L and eta_N = eta_{N-2} + 2h phi_R leaves
// [4 2; 1 4 1; ...; 2 4] eta = 6 phi + 2h (phi_L e_0 - phi_R e_{N-1}).  The interface
// slopes are then linear in (phi, phi_L, phi_R); their data part is the Neumann rows,
// and eL[q], eR[q] are the coefficients of phi_L and phi_R (at the two line ends the
// slope is the given one: eL = 1 at I = 0, eR = 1 at I = N-1).
bool hermite_end_columns(int N, double h, const std::vector<int>& ifaces, std::vector<double>& eL,
                         std::vector<double>& eR)
{
    if (N < 2 || !(h > 0.0)) return false;
    std::vector<double> cp(N), den(N), y(N), eta(N + 2);
    for (int i = 0; i < N; ++i) {
        const double sub = i == N - 1 ? 2.0 : 1.0, sup = i == 0 ? 2.0 : 1.0;
        den[i] = 4.0 - (i > 0 ? sub * cp[i - 1] : 0.0);
        cp[i] = sup / den[i];
    }
    eL.assign(ifaces.size(), 0.0);
    eR.assign(ifaces.size(), 0.0);
    for (int side = 0; side < 2; ++side) {
        // right-hand side of the unit end slope: 2h e_0 (left) or -2h e_{N-1} (right)
        for (int i = 0; i < N; ++i) {
            const double sub = i == N - 1 ? 2.0 : 1.0;
            const double r = side == 0 ? (i == 0 ? 2.0 * h : 0.0) : (i == N - 1 ? -2.0 * h : 0.0);
            y[i] = (r - (i > 0 ? sub * y[i - 1] : 0.0)) / den[i];
        }
        for (int i = N - 2; i >= 0; --i) y[i] -= cp[i] * y[i + 1];
        for (int i = 0; i < N; ++i) eta[i + 1] = y[i];
        eta[0] = eta[2] - 2.0 * h * (side == 0 ? 1.0 : 0.0);          // eta_{-1}
        eta[N + 1] = eta[N - 1] + 2.0 * h * (side == 1 ? 1.0 : 0.0);  // eta_N
        for (size_t q = 0; q < ifaces.size(); ++q) {
            const int I = ifaces[q];
            (side == 0 ? eL : eR)[q] = (eta[I + 2] - eta[I]) / (2.0 * h);
        }
    }
    return true;
}

void patch_factors(int m, double* inv, double* ainv, double* cp)
{
    double prev = 0.0;
    for (int i = 0; i <= m; ++i) {
        const double a = (i == 0) ? 0.0 : (i == m ? 1.0 / 3.0 : 1.0 / 6.0);
        const double c = (i == m) ? 0.0 : (i == 0 ? 1.0 / 3.0 : 1.0 / 6.0);
        const double den = 2.0 / 3.0 - a * prev;
        inv[i] = 1.0 / den;
        ainv[i] = a / den;
        cp[i] = c / den;
        prev = cp[i];
    }
}

// Minimum-norm correction of one stencil row so that it differentiates cubics
// exactly: sum_j c_j (j-I)^q = delta_{q1}/h, q = 0..3.  With V_jq = ((j-I)/g)^q the
// conditions read V^T c = e, e = (0, 1/(g h), 0, 0); the correction is
// delta = V (V^T V)^{-1} (e - V^T c) = Q R^{-T} (e - V^T c) for V = QR, computed by
// modified Gram-Schmidt with one re-orthogonalisation pass.
static bool cubic_exact_correction(int N, int I, int g, double h, std::vector<double>& row)
{
    const int lo = I - g < 0 ? 0 : I - g, hi = I + g > N - 1 ? N - 1 : I + g;
    const int n = hi - lo + 1;
    if (n < 4) return false;
    std::vector<double> Q((size_t)n * 4);
    double R[4][4] = {};
    for (int j = 0; j < n; ++j) {
        const double t = (double)(lo + j - I) / g;
        Q[(size_t)j * 4 + 0] = 1.0;
        Q[(size_t)j * 4 + 1] = t;
        Q[(size_t)j * 4 + 2] = t * t;
        Q[(size_t)j * 4 + 3] = t * t * t;
    }
    double r[4] = {0.0, 1.0 / (g * h), 0.0, 0.0};
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 4; ++a) r[a] -= Q[(size_t)j * 4 + a] * row[lo + j];
    for (int k = 0; k < 4; ++k) {
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < k; ++i) {
                double dot = 0.0;
                for (int j = 0; j < n; ++j) dot += Q[(size_t)j * 4 + i] * Q[(size_t)j * 4 + k];
                R[i][k] += dot;
                for (int j = 0; j < n; ++j) Q[(size_t)j * 4 + k] -= dot * Q[(size_t)j * 4 + i];
            }
        double nrm = 0.0;
        for (int j = 0; j < n; ++j) nrm += Q[(size_t)j * 4 + k] * Q[(size_t)j * 4 + k];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) return false;
        R[k][k] = nrm;
        for (int j = 0; j < n; ++j) Q[(size_t)j * 4 + k] /= nrm;
    }
    double z[4];
    for (int i = 0; i < 4; ++i) {              // R^T z = r
        double sacc = r[i];
        for (int m = 0; m < i; ++m) sacc -= R[m][i] * z[m];
        z[i] = sacc / R[i][i];
    }
    for (int j = 0; j < n; ++j) {
        double dlt = 0.0;
        for (int a = 0; a < 4; ++a) dlt += Q[(size_t)j * 4 + a] * z[a];
        row[lo + j] += dlt;
    }
    return true;
}

// Weights b1..b4 of eq. 3.8 at shift a in [0, 1].
static void weights_eq38(double a, double b[4])
{
    const double u = 1.0 - a;
    b[0] = u * u * u / 6.0;
    b[1] = -u * u * u / 2.0 + u * u / 2.0 + u / 2.0 + 1.0 / 6.0;
    b[2] = -a * a * a / 2.0 + a * a / 2.0 + a / 2.0 + 1.0 / 6.0;
    b[3] = a * a * a / 6.0;
}

bool build_axis_tables(int N, int M, int g, int G, double h, int closure, int nk, double k_lo, double hk,
                       double dt, AxisTables& out, std::string& err, double slope_lo, double slope_hi)
{
    if (N < 2 || M < 1 || g < 1 || G < g || !(h > 0.0) || nk < 1) {
        err = "axis tables: bad shape";
        return false;
    }
    out.N = N;
    out.M = M;
    out.P = npatch(N, M);
    out.MLAST = N - 1 - (out.P - 1) * M;
    out.g = g;
    out.G = G;
    out.h = h;
    const int P = out.P, W = 2 * G + 1;

    std::vector<int> ifaces(P + 1);
    for (int q = 0; q <= P; ++q) ifaces[q] = q < P ? q * M : N - 1;
    std::vector<double> rows;
    const bool hermite_rows = closure == 2 || closure == 3;
    if (!(hermite_rows ? neumann_slope_rows(N, h, ifaces, rows) : natural_slope_rows(N, h, ifaces, rows))) {
        err = "axis tables: global spline solve failed";
        return false;
    }
    out.stencil.assign((size_t)(P + 1) * W, 0.0);
    for (int q = 0; q <= P; ++q) {
        const int I = ifaces[q];
        std::vector<double> row(N, 0.0);
        for (int j = 0; j < N; ++j)
            if (std::abs(j - I) <= g) row[j] = rows[(size_t)q * N + j];
        if (closure == 1 && !cubic_exact_correction(N, I, g, h, row)) {
            err = "axis tables: cubic-exact closure needs at least 4 stencil nodes (ghost >= 3)";
            return false;
        }
        for (int j = 0; j < N; ++j) {
            if (std::abs(j - I) > g) continue;
            out.stencil[(size_t)q * W + (j - I + G)] = row[j];
        }
    }

    out.bias.assign((size_t)(P + 1), 0.0);
    if (closure == 3) {
        std::vector<double> eL, eR;
        if (!hermite_end_columns(N, h, ifaces, eL, eR)) {
            err = "axis tables: Hermite end columns failed";
            return false;
        }
        for (int q = 0; q <= P; ++q) {
            const int I = ifaces[q];
            // the given slopes sit one cell beyond the line ends (columns -1 and N):
            // kept when within the ghost width of the interface
            if (I + 1 <= g) out.bias[q] += eL[q] * slope_lo;
            if (N - I <= g) out.bias[q] += eR[q] * slope_hi;
        }
    }
    out.shift.assign(nk, 0);
    out.w.assign((size_t)nk * 4, 0.0);
    for (int i = 0; i < nk; ++i) {
        const double k = k_lo + i * hk;
        const double alpha = k * dt / h;
        double sig = std::floor(-alpha);
        double beta = -alpha - sig;
        if (beta >= 1.0) { beta -= 1.0; sig += 1.0; }
        if (beta < 0.0) beta = 0.0;
        const double lim = (double)N + 8.0;
        if (sig > lim) sig = lim;
        if (sig < -lim) sig = -lim;
        out.shift[i] = (int)sig;
        double b[4];
        weights_eq38(1.0 - beta, b);
        // cell-value taps (eta_{c-1}, eta_c, eta_{c+1}, eta_{c+2}) = (b4, b3, b2, b1)
        out.w[(size_t)i * 4 + 0] = b[3];
        out.w[(size_t)i * 4 + 1] = b[2];
        out.w[(size_t)i * 4 + 2] = b[1];
        out.w[(size_t)i * 4 + 3] = b[0];
    }
    return true;
}

}  // namespace chasm
