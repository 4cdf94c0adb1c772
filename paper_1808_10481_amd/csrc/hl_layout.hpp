// hl_layout.hpp - compile-time shapes of the Hermite-leapfrog operators.
//
// Shared by the host table builder (hl_api.cpp) and the HIP kernels so that
// both walk the packed operator tables in the same order.
//
// Per cell the method interpolates 2^d corner blocks of (m+1)^d scaled data
// into a polynomial of degree 2m+1 per variable (Sec. 2, eq. (interp); Sec. 5)
// and applies the Cauchy-Kowalevsky leapfrog weights (Sec. 2, eq. (final1);
// Sec. 3.1.2, eqs. (pdup), (vdup)).  The kernels do the interpolation of all
// but the last dimension explicitly ("slice passes") and fuse the last
// dimension's interpolation with the weight table into one "merged" table,
// so the (2m+2)^d interpolant never exists as a whole.
#pragma once

namespace hl {

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Digit k (0 = fastest) of x written in base B.
constexpr int digit(int x, int B, int k) {
  for (int i = 0; i < k; ++i) x /= B;
  return x % B;
}

template <int D, int M>
struct Dims {
  static constexpr int MP = M + 1;            // data per dimension per node
  static constexpr int N2 = 2 * M + 2;        // interpolant coefficients per dimension
  static constexpr int NC = ipow(MP, D);      // data per node per field
  static constexpr int NSL = ipow(MP, D - 1); // data per corner inside a slice
  static constexpr int NB = ipow(N2, D - 1);  // slice result: transverse coefficients
  static constexpr int NCOR = 1 << (D - 1);   // corners inside a slice
};

// Structural nonzero pattern of a merged table.  Entry (s, b) couples output
// coefficient s (in {0..m}^d) with transverse interpolant coefficient b (in
// {0..2m+1}^{d-1}).  The weight operator sum_k w_k kappa^.. Lap^k (times D_i
// for a velocity component i) moves every index down by an even amount (plus
// one in dimension i), so b_k - s_k - [k == i] must be even and >= 0.
// deriv_dim = -1: no derivative inside the table (the pressure half-step
// folds its divergence into the slice passes).
template <int D, int M>
constexpr bool merged_valid(int deriv_dim, int s, int b) {
  for (int k = 0; k < D - 1; ++k) {
    const int sk = digit(s, M + 1, k);
    const int bk = digit(b, 2 * M + 2, k);
    const int r = bk - sk - (deriv_dim == k ? 1 : 0);
    if (r < 0 || (r & 1)) return false;
  }
  return true;
}

template <int D, int M>
constexpr int merged_nnz(int deriv_dim) {
  int n = 0;
  for (int s = 0; s < Dims<D, M>::NC; ++s)
    for (int b = 0; b < Dims<D, M>::NB; ++b)
      if (merged_valid<D, M>(deriv_dim, s, b)) ++n;
  return n;
}

// Packed merged table for one group: for eL in {0,1} (last-dimension corner),
// l in {0..m} (last-dimension datum), then (s, b) valid in row-major order.
template <int D, int M>
constexpr int merged_size(int deriv_dim) {
  return 2 * (M + 1) * merged_nnz<D, M>(deriv_dim);
}

// Pass tables: kind 0 = H (interpolation, 2m+2 rows), kind 1 + k = D_k H
// (x_k-derivative of the interpolant; last row zero).  Each is (2m+2) x (m+1)
// and acts on sigma_l = R_l + L_l / delta_l = R_l - L_l: row b uses sigma_l
// when b + l + flip is even, delta_l otherwise (flip = 1 for D_k H), which is
// the xi -> -xi symmetry of the interpolant.
template <int D, int M>
struct TableLayout {
  static constexpr int PASS = (2 * M + 2) * (M + 1);   // one pass table
  static constexpr int NPASS = 1 + D;                  // H, D_1 H, .., D_d H
  static constexpr int PASS_OFF = 0;
  // pressure half-step groups: A = components 0..d-2 (last pass H),
  // B = component d-1 (last pass D_d H); both without derivative in the table
  static constexpr int PG = merged_size<D, M>(-1);
  static constexpr int P_A_OFF = PASS_OFF + NPASS * PASS;
  static constexpr int P_B_OFF = P_A_OFF + (D > 1 ? PG : 0);
  // velocity half-step: one table per output component i (derivative D_i)
  static constexpr int U_OFF = P_B_OFF + PG;
  static constexpr int u_size(int i) { return merged_size<D, M>(i); }
  static constexpr int u_off(int i) {
    int o = U_OFF;
    for (int k = 0; k < i; ++k) o += merged_size<D, M>(k);
    return o;
  }
  static constexpr int TOTAL = u_off(D);
};

}  // namespace hl
