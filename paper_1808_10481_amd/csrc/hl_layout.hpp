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
// Velocity outputs through one scalar polynomial.  Every velocity increment
// is a derivative of the same polynomial Q = sum_k w_k kappa^k Lap^k c
// (Sec. 3.1.2, eq. (vdup): u_i picks up D_i Lap^k), so
//   u_i[s] -= (s_i + 1) / h_i * Q[s + e_i],   s in {0..m}^d.
// The kernels accumulate Q only on the index set
//   G = { s' in {0..m+1}^d : s' - e_i in {0..m}^d for some i }
// (all of {0..m}^d except 0, plus the points with exactly one coordinate
// m+1), |G| = (m+1)^d - 1 + d (m+1)^{d-1}: 53 values for d = 3, m = 2 against
// 3 x 27 velocity outputs, with fewer table terms as well.
// ---------------------------------------------------------------------------
template <int D, int M>
struct GSet {
  static constexpr int count() {
    int n = 0;
    for (int x = 0; x < ipow(M + 2, D); ++x) {
      int top = 0, nz = 0;
      for (int k = 0; k < D; ++k) {
        const int v = digit(x, M + 2, k);
        if (v == M + 1) ++top;
        if (v != 0) ++nz;
      }
      if (top <= 1 && nz > 0) ++n;
    }
    return n;
  }
  static constexpr int NG = count();
  int dig[NG][D > 0 ? D : 1];   // digits of each member, dimension 0 first
  constexpr GSet() : dig() {
    int n = 0;
    for (int x = 0; x < ipow(M + 2, D); ++x) {
      int top = 0, nz = 0;
      for (int k = 0; k < D; ++k) {
        const int v = digit(x, M + 2, k);
        if (v == M + 1) ++top;
        if (v != 0) ++nz;
      }
      if (top <= 1 && nz > 0) {
        for (int k = 0; k < D; ++k) dig[n][k] = digit(x, M + 2, k);
        ++n;
      }
    }
  }
  // member index of s' (digits), or -1
  constexpr int find(const int* sd) const {
    for (int g = 0; g < NG; ++g) {
      bool eq = true;
      for (int k = 0; k < D; ++k) eq = eq && dig[g][k] == sd[k];
      if (eq) return g;
    }
    return -1;
  }
};

template <int D, int M>
inline constexpr GSet<D, M> kGSet{};

// ---------------------------------------------------------------------------
// Merged tables.  Entry (l, o, b): last-dimension datum l, output o (a
// pressure coefficient s in {0..m}^d, or a member s' of G for the velocity),
// transverse interpolant coefficient b in {0..2m+1}^{d-1}:
//   M[l][o][b] = sum_{b_L} W(o, (b, b_L)) G_last[b_L][l]
// where W is the weight operator sum_k w_k kappa^.. Lap^k and G_last the last
// dimension's pass table.  Lap moves every index down by an even amount, so
// the entry is structurally nonzero only when b_k - o_k is even and >= 0 for
// every transverse k.  All contributing b_L share the parity of o_L, so the
// entry multiplies sigma_l or delta_l of the two last-dimension corners as
// (o_L + l + flip_last) is even or odd.
// ---------------------------------------------------------------------------
template <int D, int M>
constexpr bool out_digits(bool velocity, int o, int* od) {
  if (!velocity) {
    for (int k = 0; k < D; ++k) od[k] = digit(o, M + 1, k);
  } else {
    for (int k = 0; k < D; ++k) od[k] = kGSet<D, M>.dig[o][k];
  }
  return true;
}

template <int D, int M>
constexpr int n_out(bool velocity) {
  return velocity ? GSet<D, M>::NG : Dims<D, M>::NC;
}

template <int D, int M>
constexpr bool merged_valid(bool velocity, int o, int b) {
  int od[3] = {0, 0, 0};
  out_digits<D, M>(velocity, o, od);
  for (int k = 0; k < D - 1; ++k) {
    const int r = digit(b, 2 * M + 2, k) - od[k];
    if (r < 0 || (r & 1)) return false;
  }
  return true;
}

template <int D, int M>
constexpr bool merged_uses_delta(bool velocity, int flip_last, int o, int l) {
  int od[3] = {0, 0, 0};
  out_digits<D, M>(velocity, o, od);
  return ((od[D - 1] + l + flip_last) & 1) != 0;
}

template <int D, int M>
constexpr int merged_nnz(bool velocity) {
  int n = 0;
  for (int o = 0; o < n_out<D, M>(velocity); ++o)
    for (int b = 0; b < Dims<D, M>::NB; ++b)
      if (merged_valid<D, M>(velocity, o, b)) ++n;
  return n;
}

// Packed merged table for one group: l in {0..m}, then the valid (o, b) in
// row-major order.
template <int D, int M>
constexpr int merged_size(bool velocity) {
  return (M + 1) * merged_nnz<D, M>(velocity);
}

// Compile-time walk of one merged table: entry t multiplies input b[t] into
// output o[t]; base_delta[o] is the sigma/delta selector for l = 0 (it flips
// with the parity of l).  Used by the kernels so every index is a constant
// after unrolling.
template <int D, int M, bool VEL, int FLIPL>
struct MergeSpec {
  static constexpr int NNZ = merged_nnz<D, M>(VEL);
  static constexpr int NO = n_out<D, M>(VEL);
  short o[NNZ];
  short b[NNZ];
  bool base_delta[NO];
  constexpr MergeSpec() : o(), b(), base_delta() {
    int t = 0;
    for (int oo = 0; oo < NO; ++oo) {
      base_delta[oo] = merged_uses_delta<D, M>(VEL, FLIPL, oo, 0);
      for (int bb = 0; bb < Dims<D, M>::NB; ++bb)
        if (merged_valid<D, M>(VEL, oo, bb)) {
          o[t] = (short)oo;
          b[t] = (short)bb;
          ++t;
        }
    }
  }
};

template <int D, int M, bool VEL, int FLIPL>
inline constexpr MergeSpec<D, M, VEL, FLIPL> kMerge{};

// Member of G holding Q[s + e_i] for velocity component i and coefficient s.
template <int D, int M>
struct GIndex {
  short g[D][Dims<D, M>::NC];
  constexpr GIndex() : g() {
    for (int i = 0; i < D; ++i)
      for (int s = 0; s < Dims<D, M>::NC; ++s) {
        int sd[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) sd[k] = digit(s, M + 1, k);
        sd[i] += 1;
        g[i][s] = (short)kGSet<D, M>.find(sd);
      }
  }
};

template <int D, int M>
inline constexpr GIndex<D, M> kGIndex{};

// ---------------------------------------------------------------------------
// 3D: interpolation is explicit only along x; y and z are merged into the
// table.  For y/z data a' = (a_y, a_z) and output o:
//   M[a'][o][b_x] = scale * sum_{b_y, b_z} W(o, b) Gy[b_y][a_y] Gz[b_z][a_z]
// acting on the combination of the four (y, z) corners' x-interpolants
//   X[k_y][k_z] = sum_{e_y, e_z} (+-1) Y_{e_y e_z},  k = sigma (R + L) or delta (R - L),
// with k_y = sigma iff o_y + a_y + flip_y is even (likewise z).  Structural
// nonzeros: b_x - o_x even and >= 0.  Walk order: a' block, then o, then b_x.
// ---------------------------------------------------------------------------
template <int M>
constexpr int count_bx(int ox) {
  int n = 0;
  for (int bx = ox; bx < 2 * M + 2; bx += 2) ++n;
  return n;
}

template <int M, bool VEL>
constexpr int merge3_block_nnz() {
  int n = 0;
  for (int o = 0; o < n_out<3, M>(VEL); ++o) {
    int od[3] = {0, 0, 0};
    out_digits<3, M>(VEL, o, od);
    n += count_bx<M>(od[0]);
  }
  return n;
}

template <int M, bool VEL>
constexpr int merge3_size() {
  return (M + 1) * (M + 1) * merge3_block_nnz<M, VEL>();
}

template <int M, bool VEL, int FY, int FZ>
struct Merge3Spec {
  static constexpr int NNZ = merge3_block_nnz<M, VEL>();  // per a' block
  short o[NNZ];
  short bx[NNZ];
  unsigned char ky[NNZ][M + 1];  // 1 = delta in y, for a_y
  unsigned char kz[NNZ][M + 1];  // 1 = delta in z, for a_z
  constexpr Merge3Spec() : o(), bx(), ky(), kz() {
    int t = 0;
    for (int oo = 0; oo < n_out<3, M>(VEL); ++oo) {
      int od[3] = {0, 0, 0};
      out_digits<3, M>(VEL, oo, od);
      for (int b = od[0]; b < 2 * M + 2; b += 2) {
        o[t] = (short)oo;
        bx[t] = (short)b;
        for (int a = 0; a <= M; ++a) {
          ky[t][a] = (unsigned char)((od[1] + a + FY) & 1);
          kz[t][a] = (unsigned char)((od[2] + a + FZ) & 1);
        }
        ++t;
      }
    }
  }
};

template <int M, bool VEL, int FY, int FZ>
inline constexpr Merge3Spec<M, VEL, FY, FZ> kMerge3{};

template <int D, int M>
struct TableLayout;

// 1D / 2D: pressure groups per component (the last one carries the
// derivative pass of the last dimension), then the velocity (Q) table.
template <int D, int M>
struct TableLayout {
  static constexpr int PG = merged_size<D, M>(false);
  static constexpr int P_A_OFF = 0;                          // component 0 (2D)
  static constexpr int P_B_OFF = P_A_OFF + (D > 1 ? PG : 0); // component d-1
  static constexpr int U_OFF = P_B_OFF + PG;
  static constexpr int TOTAL = U_OFF + merged_size<D, M>(true);
  static constexpr int p_off(int i) { return (D > 1 && i == 0) ? P_A_OFF : P_B_OFF; }
};

// 3D: one pressure table per component (derivative dimension), then Q (the
// (y, z) merged tables of the explicit x-pass path); then the fully merged
// pressure table (x merged too): F[i][a][o], component i, datum a, output o,
// (m+1)^3 x (m+1)^3 per component, and the fully merged velocity table
// Fu[a][o] over the members o of G.  The kernels use the fully merged tables
// (one FMA per entry after the corner butterfly) for every m;
// HL_FULLP_MAXM / HL_FULLU_MAXM below 3 select the explicit x pass plus the
// (y, z) tables for the larger m instead (at m = 3 that path needs 512 VGPRs
// and spills 1.8-2.6 KB per lane).
#ifndef HL_FULLP_MAXM
#define HL_FULLP_MAXM 3
#endif
#ifndef HL_FULLU_MAXM
#define HL_FULLU_MAXM 3
#endif

template <int M>
struct TableLayout<3, M> {
  static constexpr int PG = merge3_size<M, false>();
  static constexpr int p_off(int i) { return i * PG; }
  static constexpr int P_A_OFF = 0;
  static constexpr int P_B_OFF = 2 * PG;
  static constexpr int U_OFF = 3 * PG;
  static constexpr bool FULL_P = M <= HL_FULLP_MAXM;
  static constexpr int NC = (M + 1) * (M + 1) * (M + 1);
  static constexpr int F_OFF = U_OFF + merge3_size<M, true>();
  // the fully merged velocity table Fu[a][o], datum a, member o of G
  static constexpr bool FULL_U = M <= HL_FULLU_MAXM;
  static constexpr int FU_OFF = F_OFF + (FULL_P ? 3 * NC * NC : 0);
  static constexpr int TOTAL = FU_OFF + (FULL_U ? NC * GSet<3, M>::NG : 0);
};

}  // namespace hl
