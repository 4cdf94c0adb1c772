// hl_layout.hpp - compile-time shapes of the Hermite-leapfrog operators.
//
// Shared by the host table builder (hl_api.hip) and the HIP kernels so that
// both walk the packed operator tables in the same order.
//
// Per cell the method interpolates 2^d corner blocks of (m+1)^d scaled data
// into a polynomial of degree 2m+1 per variable (Sec. 2, eq. (interp); Sec. 5)
// and applies the Cauchy-Kowalevsky leapfrog weights (Sec. 2, eq. (final1);
// Sec. 3.1.2, eqs. (pdup), (vdup)).  The kernels interpolate all but the last
// dimension explicitly ("slice passes", compile-time constants) and fuse the
// last dimension's interpolation with the weight operator into one runtime
// "merged" table, so the (2m+2)^d interpolant never exists as a whole.
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
  static constexpr int NB = ipow(N2, D - 1);  // slice result: transverse coefficients
};

// ---------------------------------------------------------------------------
// Exact Hermite-Birkhoff matrix at compile time (Sec. 2, eq. (interp)):
// H = [C^L; C^R]^{-1}, C_{ls} = binom(s, l) xi0^{s-l}, xi0 = -1/2 (left),
// +1/2 (right).  By the xi -> -xi symmetry H[s][L_l] = (-1)^{s+l} H[s][R_l],
// so c_s = sum_l H[s][R_l] * (R_l + (-1)^{s+l} L_l): row s uses
// sigma_l = R_l + L_l when s + l is even and delta_l = R_l - L_l otherwise.
// g[s][l] = H[s][R_l] in exact rationals, rounded once to double.
// ---------------------------------------------------------------------------
struct CRat {
  long long n, d;
};
constexpr long long cgcd(long long a, long long b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) {
    const long long t = a % b;
    a = b;
    b = t;
  }
  return a ? a : 1;
}
constexpr CRat crat(long long n, long long d) {
  if (d < 0) n = -n, d = -d;
  const long long g = cgcd(n, d);
  return CRat{n / g, d / g};
}
constexpr CRat cmul(CRat a, CRat b) { return crat(a.n * b.n, a.d * b.d); }
constexpr CRat csub(CRat a, CRat b) { return crat(a.n * b.d - b.n * a.d, a.d * b.d); }
constexpr CRat cdiv(CRat a, CRat b) { return crat(a.n * b.d, a.d * b.n); }
constexpr long long cbinom(int n, int k) {
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

template <int M>
struct HermiteConst {
  static constexpr int MP = M + 1, N2 = 2 * M + 2;
  double g[N2][MP];
  constexpr HermiteConst() : g() {
    CRat A[N2][2 * N2] = {};
    for (int r = 0; r < N2; ++r)
      for (int c = 0; c < 2 * N2; ++c) A[r][c] = CRat{0, 1};
    for (int side = 0; side < 2; ++side)
      for (int l = 0; l <= M; ++l)
        for (int s = l; s < N2; ++s) {
          CRat pw{1, 1};
          for (int q = 0; q < s - l; ++q) pw = cmul(pw, CRat{side ? 1 : -1, 2});
          A[side * MP + l][s] = cmul(CRat{cbinom(s, l), 1}, pw);
        }
    for (int r = 0; r < N2; ++r) A[r][N2 + r] = CRat{1, 1};
    for (int col = 0; col < N2; ++col) {
      int piv = col;
      while (A[piv][col].n == 0) ++piv;
      for (int c = 0; c < 2 * N2; ++c) {
        const CRat t = A[piv][c];
        A[piv][c] = A[col][c];
        A[col][c] = t;
      }
      const CRat pv = A[col][col];
      for (int c = 0; c < 2 * N2; ++c) A[col][c] = cdiv(A[col][c], pv);
      for (int r = 0; r < N2; ++r) {
        if (r == col || A[r][col].n == 0) continue;
        const CRat f = A[r][col];
        for (int c = 0; c < 2 * N2; ++c) A[r][c] = csub(A[r][c], cmul(f, A[col][c]));
      }
    }
    for (int s = 0; s < N2; ++s)
      for (int l = 0; l < MP; ++l) g[s][l] = (double)A[s][N2 + MP + l].n / (double)A[s][N2 + MP + l].d;
  }
};

template <int M>
inline constexpr HermiteConst<M> kHermite{};

// Coefficient of a slice pass.  FLIP = 0: interpolation H (rows b = 0..2m+1);
// FLIP = 1: x-derivative of the interpolant in units of 1/h, (b+1) H[b+1]
// (rows b = 0..2m; row 2m+1 is zero).  Row b uses sigma_l when b + l + FLIP
// is even, delta_l otherwise.
template <int M, int FLIP>
constexpr double pass_coef(int b, int l) {
  if (FLIP == 0) return kHermite<M>.g[b][l];
  return (b + 1 < 2 * M + 2) ? (double)(b + 1) * kHermite<M>.g[b + 1][l] : 0.0;
}

// ---------------------------------------------------------------------------
// Merged tables.  Entry (l, s, b): last-dimension datum l, output coefficient
// s in {0..m}^d, transverse interpolant coefficient b in {0..2m+1}^{d-1}:
//   M[l][s][b] = sum_{b_L} W(s, (b, b_L)) G_last[b_L][l]
// where W is the weight operator (sum_k w_k kappa^.. Lap^k, times D_i for a
// velocity component i) and G_last the last dimension's pass table.  W moves
// every index down by an even amount (plus one in dimension i), so the entry
// is structurally nonzero only when b_k - s_k - [k == i] is even and >= 0 for
// every transverse k.  All contributing b_L share the parity of s_L + [i last],
// so the entry multiplies sigma_l or delta_l of the two last-dimension corners
// as (s_L + [i last] + l + flip_last) is even or odd.
// deriv_dim = -1: no derivative inside W (pressure: the divergence is folded
// into the slice passes and the last pass).
// ---------------------------------------------------------------------------
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
constexpr bool merged_uses_delta(int deriv_dim, int flip_last, int s, int l) {
  const int sL = digit(s, M + 1, D - 1);
  return ((sL + (deriv_dim == D - 1 ? 1 : 0) + l + flip_last) & 1) != 0;
}

template <int D, int M>
constexpr int merged_nnz(int deriv_dim) {
  int n = 0;
  for (int s = 0; s < Dims<D, M>::NC; ++s)
    for (int b = 0; b < Dims<D, M>::NB; ++b)
      if (merged_valid<D, M>(deriv_dim, s, b)) ++n;
  return n;
}

// Packed merged table for one group: l in {0..m}, then the valid (s, b) in
// row-major order.
template <int D, int M>
constexpr int merged_size(int deriv_dim) {
  return (M + 1) * merged_nnz<D, M>(deriv_dim);
}

template <int D, int M>
struct TableLayout {
  // pressure half-step groups: A = components 0..d-2 (last pass H),
  // B = component d-1 (last pass D_d H); W without derivative
  static constexpr int PG = merged_size<D, M>(-1);
  static constexpr int P_A_OFF = 0;
  static constexpr int P_B_OFF = P_A_OFF + (D > 1 ? PG : 0);
  // velocity half-step: one table per output component i (W with D_i)
  static constexpr int U_OFF = P_B_OFF + PG;
  static constexpr int u_off(int i) {
    int o = U_OFF;
    for (int k = 0; k < i; ++k) o += merged_size<D, M>(k);
    return o;
  }
  static constexpr int TOTAL = u_off(D);
};

}  // namespace hl
