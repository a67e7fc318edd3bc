// chasm_tables.hpp -- host-side FP64 tables of one axis of the advection step.
//
// For an axis of N nodes with patches of M cells, ghost width g, spacing h:
//   stencil  (P+1) rows of width 2G+1: interface slopes d_q = sum_t S[q][t] phi[I_q-G+t]
//            (PMBC, eqs. 3.4-3.5; rows of the natural-BC inverse, truncated to
//            |j - I_q| <= g; G >= g is the window).  The kernels carry the same rows
//            (times h) as compile-time constants; this FP64 copy is the host record
//            the tests compare them with.
//   shift/w  per k node: sigma = floor(-alpha), alpha = k dt / h, and the weights
//            w_r = b_{4-r}(1 - beta) of eq. 3.8, beta = -alpha - sigma.
#pragma once
#include <string>
#include <vector>

namespace chasm {

struct AxisTables {
    int N = 0, M = 0, P = 0, MLAST = 0, g = 0, G = 0;
    double h = 0.0;
    std::vector<double> stencil;   // (P+1)*(2G+1)
    std::vector<int> shift;        // nk
    std::vector<double> w;         // nk*4
    std::vector<double> bias;      // P+1: slope part from the given end slopes (closure 3)
};

// Number of patches of M cells covering N nodes.
inline int npatch(int N, int M) { return (N - 1 + M - 1) / M; }

// Slopes s'(x_I) of the natural cubic spline of the data, as rows over the data:
// out[(N)*q + j] for each requested interface I_q.  Returns false on bad input.
bool natural_slope_rows(int N, double h, const std::vector<int>& ifaces, std::vector<double>& out);

// The same for the Neumann global spline (zero slopes at both ends).
bool neumann_slope_rows(int N, double h, const std::vector<int>& ifaces, std::vector<double>& out);

// Coefficients of the given end slopes in the interface slopes of the Hermite global
// spline (eq. 2.13): eL[q] for phi_L, eR[q] for phi_R.
bool hermite_end_columns(int N, double h, const std::vector<int>& ifaces, std::vector<double>& eL,
                         std::vector<double>& eR);

// Thomas factors of the reduced patch system of m+1 rows (see PatchLU in chasm_line.hpp):
// inv, ainv, cp of length m+1.
void patch_factors(int m, double* inv, double* ainv, double* cp);

// Build every table of one axis.  closure: 0 paper PMBC, 1 cubic-exact variant,
// 2 Neumann global spline, 3 Hermite global spline with end slopes slope_lo, slope_hi.
bool build_axis_tables(int N, int M, int g, int G, double h, int closure, int nk, double k_lo, double hk,
                       double dt, AxisTables& out, std::string& err, double slope_lo = 0.0,
                       double slope_hi = 0.0);

}  // namespace chasm
