// hl_api.hip - C ABI of the Hermite-leapfrog library: validation, operator
// tables, host<->device layout conversion, stepping and diagnostics.
//
// Operator tables (built once per plan, FP64, then cast to the plan's
// arithmetic type):
//  * H_m = [C^L; C^R]^{-1} (Sec. 2, eq. (interp)), by exact rational
//    Gauss-Jordan elimination; C_{ls} = binom(s, l) xi0^{s-l}, xi0 = -+1/2.
//  * the weight operators of the leapfrog difference with Cauchy-Kowalevsky
//    exchange (Sec. 2, eqs. (update1), (final1); Sec. 3.1.2, eqs. (pdup),
//    (vdup)): with w_k = 2 (dt/2)^{2k+1} / (2k+1)!,
//      pressure:   W_p   = sum_k w_k kappa^{k+1} Lap^k      (divergence folded
//                                                            into the passes)
//      velocity i: W_u,i = sum_k w_k kappa^k D_i Lap^k
//    as coefficient-space operators on the cell polynomial, restricted to
//    output coefficients s in {0..m}^d (the new nodal data are the Taylor
//    coefficients at the node, Sec. 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <array>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hl.h"
#include "hl_host_layout.hpp"
#include "hl_internal.hpp"

namespace {

thread_local std::string g_last_error;

hl_status fail(hl_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

hl_status hip_fail(hipError_t e, const char* where) {
  return fail(HL_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Exact rationals for H_m (entries are small; __int128 with gcd reduction).
// ---------------------------------------------------------------------------
struct Rat {
  __int128 n = 0, d = 1;
};
__int128 gcd128(__int128 a, __int128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) {
    __int128 t = a % b;
    a = b;
    b = t;
  }
  return a ? a : 1;
}
Rat mk(__int128 n, __int128 d) {
  if (d < 0) n = -n, d = -d;
  const __int128 g = gcd128(n, d);
  return Rat{n / g, d / g};
}
Rat add(Rat a, Rat b) { return mk(a.n * b.d + b.n * a.d, a.d * b.d); }
Rat sub(Rat a, Rat b) { return mk(a.n * b.d - b.n * a.d, a.d * b.d); }
Rat mul(Rat a, Rat b) { return mk(a.n * b.n, a.d * b.d); }
Rat dvd(Rat a, Rat b) { return mk(a.n * b.d, a.d * b.n); }
double to_double(Rat a) { return (double)(long double)a.n / (double)(long double)a.d; }

long long binom(int n, int k) {
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// H[s][col], s = 0..2m+1, col = (L_0..L_m, R_0..R_m).
std::vector<double> hermite_matrix(int m) {
  const int n = 2 * m + 2;
  std::vector<Rat> A(n * 2 * n);
  for (int side = 0; side < 2; ++side) {
    const Rat xi0 = mk(side ? 1 : -1, 2);
    for (int l = 0; l <= m; ++l)
      for (int s = l; s < n; ++s) {
        Rat pw = mk(1, 1);
        for (int q = 0; q < s - l; ++q) pw = mul(pw, xi0);
        A[(side * (m + 1) + l) * 2 * n + s] = mul(mk(binom(s, l), 1), pw);
      }
  }
  for (int r = 0; r < n; ++r) A[r * 2 * n + n + r] = mk(1, 1);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    while (A[piv * 2 * n + col].n == 0) ++piv;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) std::swap(A[piv * 2 * n + c], A[col * 2 * n + c]);
    const Rat pv = A[col * 2 * n + col];
    for (int c = 0; c < 2 * n; ++c) A[col * 2 * n + c] = dvd(A[col * 2 * n + c], pv);
    for (int r = 0; r < n; ++r) {
      if (r == col || A[r * 2 * n + col].n == 0) continue;
      const Rat f = A[r * 2 * n + col];
      for (int c = 0; c < 2 * n; ++c) A[r * 2 * n + c] = sub(A[r * 2 * n + c], mul(f, A[col * 2 * n + c]));
    }
  }
  std::vector<double> H(n * n);
  for (int s = 0; s < n; ++s)
    for (int c = 0; c < n; ++c) H[s * n + c] = to_double(A[s * 2 * n + n + c]);
  return H;
}

// ---------------------------------------------------------------------------
// Coefficient-space polynomial operators on (2m+2)^d dense arrays, index
// b = b_1 + N2 (b_2 + N2 b_3).
// ---------------------------------------------------------------------------
struct PolyOps {
  int d, N2, size;
  double h[3];
  int stride(int k) const { return k == 0 ? 1 : (k == 1 ? N2 : N2 * N2); }
  int dig(int b, int k) const { return (b / stride(k)) % N2; }
  // D_k: (D_k c)_b = (b_k + 1) c_{b + e_k} / h_k
  std::vector<double> deriv(const std::vector<double>& c, int k) const {
    std::vector<double> o(size, 0.0);
    for (int b = 0; b < size; ++b) {
      const int bk = dig(b, k);
      if (bk + 1 < N2) o[b] = (bk + 1) * c[b + stride(k)] / h[k];
    }
    return o;
  }
  std::vector<double> lap(const std::vector<double>& c) const {
    std::vector<double> o(size, 0.0);
    for (int k = 0; k < d; ++k) {
      std::vector<double> t = deriv(deriv(c, k), k);
      for (int b = 0; b < size; ++b) o[b] += t[b];
    }
    return o;
  }
};

bool all_zero(const std::vector<double>& v) {
  for (double x : v)
    if (x != 0.0) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct hl_plan_s {
  hl_problem prob;
  int d, m, precision, nc;
  int word_bytes;      // bytes per state word
  int words_per_coef;  // 1 (FP64, FP32) or 3 (FP32_COMP: FP32 hi + BF16 lo)
  int tab_bytes;       // bytes per table entry (arithmetic type)
  double dt, nu, kappa, h[3];
  bool walls = false;
  int32_t K[3];          // cells per dimension (1 beyond d)
  // device arrays: p with extents pext (offset 0), u with extents uext and
  // dual node q at index q + uoff (walls: one ghost node per side)
  int32_t pext[3], uext[3], uoff;
  int64_t pnodes, unodes;
  hl::Grid gp, gu;       // pressure / velocity half-step launch grids
  int32_t ygroup_req = 0; // 3D tile rows per group asked for (the grids clamp it to their extent)
  hl::KernelSet ks;
  void* dtab = nullptr;
  void* dadj = nullptr;        // adjoint blocks (B^T then A^T), or NULL
  size_t adj_u_off = 0;        // element offset of the A^T blocks in dadj
  // kappa gradient, allocated on first use: tables with kappa-derivative
  // weights and with -dt (one step reversed), copies of the forward state
  // walked back step by step, scratch fields and reduction partials
  // variable kappa (hl_set_kappa): Taylor data on the primal / dual nodes
  bool var_kappa = false;
  void* dkap_p = nullptr;
  void* dkap_u = nullptr;
  // variable-kappa adjoint (allocated on first use): FP64 gradient
  // accumulators, one plane per kappa coefficient on the primal / dual nodes,
  // and the scratch of d (2m+2)^d planes between its two kernels
  double* gkp = nullptr;
  double* gku = nullptr;
  void* vscr = nullptr;
  void* wscr = nullptr;  // walls adjoint: A^T p_bar on the padded velocity array (kept zeroed)
  void* vzw = nullptr;   // walls, variable-kappa adjoint: dS/dc on the padded dual array (ghost slots zero)
  void* ucw = nullptr;   // walls, variable-kappa adjoint: copy of U_t with its ghost layer refreshed
  void* tab_dk = nullptr;
  void* tab_rev = nullptr;
  void* fp = nullptr;
  void* fu = nullptr;
  void* sp = nullptr;
  void* su = nullptr;
  double* gpart = nullptr;
  double* dpartial = nullptr;  // norms scratch, kNormBlocks per plane
  int device = 0;
  // hl_step replays a captured graph of kGraphChunk steps for the last
  // (p, u) pair it saw; the capture runs on a plan-owned stream and the graph
  // is launched on the caller's stream.
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* graph_p = nullptr;  // buffers the graph was captured for
  const void* graph_u = nullptr;
  // bumped by every call that changes what a batch descriptor bakes in
  // (kappa buffers, launch grids): hl_set_kappa, hl_set_tile (and hl_tune)
  uint64_t gen = 0;
};

// A batch of shots (plans of the same d, m and precision) advanced together.
struct hl_batch_s {
  std::vector<hl_plan_s*> plans;
  hl::KernelSet ks;                   // the common kernel set
  int device = 0;
  bool var = false;                   // variable kappa (every plan, or none)
  void* dp = nullptr;                 // device descriptors of the p / u half-steps
  void* du = nullptr;
  size_t cap = 0;                     // bytes allocated for each
  std::vector<void*> bp, bu;          // buffers the descriptors describe
  std::vector<uint64_t> gens;         // the member plans' generations they were built at
  std::vector<hl::PlanView> views;    // per shot (walled shots: the ghost refresh)
  int32_t tile[3] = {0, 0, 0};        // workgroup shape and 3D y-group of the batched launches
  bool walls = false;                 // some shot has reflecting walls
  int pblocks = 0, ublocks = 0;
  hipStream_t cap_stream = nullptr;   // graph of kGraphChunk batched steps
  hipGraphExec_t gexec = nullptr;
  // sources (hl_batch_set_sources): entries, values and amplitudes on the
  // device, the shots' pressure buffers, and the step counter
  bool src = false;
  void* d_pbase = nullptr;
  void* d_ent = nullptr;
  void* d_val = nullptr;
  void* d_amps = nullptr;
  int64_t* d_counter = nullptr;
  int64_t nent = 0, namps = 0;
};

namespace {

constexpr int kNormBlocks = 256;
constexpr int64_t kGraphChunk = 16;   // steps per captured graph (32 kernel nodes)
#ifndef HL_3D_YGROUP
#define HL_3D_YGROUP 2
#endif
constexpr int32_t kYGroup3 = HL_3D_YGROUP;

// Advances a batch's step counter (one work-item; runs after the step's source).
__global__ void batch_tick(int64_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += 1;
}

void drop_sources(hl_batch_s* b) {
  for (void** q : {&b->d_pbase, &b->d_ent, &b->d_val, &b->d_amps, (void**)&b->d_counter}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  b->src = false;
  b->nent = b->namps = 0;
}

void drop_graph(hl_plan_s* pl) {
  if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
  pl->gexec = nullptr;
  pl->graph_p = pl->graph_u = nullptr;
}

// Half-step launchers of the plan: constant or variable kappa.
hl::PHalfFn p_fn(const hl_plan_s* pl) { return pl->var_kappa ? pl->ks.p_half_var : pl->ks.p_half; }
hl::UHalfFn u_fn(const hl_plan_s* pl) { return pl->var_kappa ? pl->ks.u_half_var : pl->ks.u_half; }

// Capture kGraphChunk steps for buffers (p, u) into pl->gexec.
hipError_t capture_steps(hl_plan_s* pl, const hl::PlanView& v, void* p, void* u) {
  hipError_t e = hipSuccess;
  if (!pl->cap_stream) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  drop_graph(pl);
  e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int64_t n = 0; n < kGraphChunk && le == hipSuccess; ++n) {
    if (pl->walls) le = pl->ks.ghost(v, u, pl->cap_stream);
    if (le == hipSuccess) le = p_fn(pl)(v, p, u, pl->cap_stream);
    if (le == hipSuccess) le = u_fn(pl)(v, u, p, 1.0, pl->cap_stream);
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(pl->cap_stream, &graph);
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&pl->gexec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e == hipSuccess) {
    pl->graph_p = p;
    pl->graph_u = u;
  } else {
    pl->gexec = nullptr;
  }
  return e;
}

int max_m(int d) { return d == 1 ? 7 : (d == 2 ? 5 : 3); }

PolyOps poly_ops(const hl_plan_s* pl) {
  PolyOps P;
  P.d = pl->d;
  P.N2 = 2 * pl->m + 2;
  P.size = 1;
  for (int k = 0; k < pl->d; ++k) P.size *= P.N2;
  for (int k = 0; k < 3; ++k) P.h[k] = pl->h[k];
  return P;
}

// Weights of the operator tables: the time step (its sign reverses a step:
// every w_k is odd in dt) and whether the kappa powers are replaced by their
// kappa-derivatives (the operators A_kappa, B_kappa of the gradient).
struct WeightMode {
  double dt;
  bool dkappa;
};

// W = sum_k w_k kappa^{k + kshift} Lap^k as a full (2m+2)^d x (2m+2)^d
// operator on cell polynomials, rows = output coefficient, w_k =
// 2 (dt/2)^{2k+1} / (2k+1)! (Sec. 2, eq. (update1); Sec. 3.1.2, eqs. (pdup),
// (vdup)); the series stops where Lap^k of the basis monomial vanishes.  With
// wm.dkappa, kappa^j becomes j kappa^{j-1}.
std::vector<double> weight_operator(const hl_plan_s* pl, const PolyOps& P, int kshift, WeightMode wm) {
  std::vector<double> W((size_t)P.size * P.size, 0.0);
  for (int beta = 0; beta < P.size; ++beta) {
    std::vector<double> term(P.size, 0.0), acc(P.size, 0.0);
    term[beta] = 1.0;
    double fact = 1.0;
    for (int k = 0; !all_zero(term); ++k) {
      if (k > 0) fact *= (double)(2 * k) * (double)(2 * k + 1);
      const int j = k + kshift;
      const double kp = wm.dkappa ? (j > 0 ? j * std::pow(pl->kappa, j - 1) : 0.0) : std::pow(pl->kappa, j);
      const double ck = 2.0 * std::pow(wm.dt / 2.0, 2 * k + 1) / fact * kp;
      for (int b = 0; b < P.size; ++b) acc[b] += ck * term[b];
      term = P.lap(term);
    }
    for (int b = 0; b < P.size; ++b) W[(size_t)b * P.size + beta] = acc[b];
  }
  return W;
}

// Dense per-corner blocks of the transposed half-steps (periodic plans),
// packed as the adjoint kernels read them: T[e'][io][ii][r][c].
//   A[e][s][i][a]: the pressure half-step subtracts A[e] U_i[j - 1 + e] from P[j]:
//     A[e][s][i][a] = sum_b Wp[s][b] (D_i I_{e,a})_b,
//   B[e][i][s][a]: the velocity half-step subtracts B[e] P[q + e] from U_i[q]:
//     B[e][i][s][a] = (s_i + 1) / h_i sum_b Wq[s + e_i][b] (I_{e,a})_b,
// with I_{e,a} the interpolant of a unit datum a at corner e (Sec. 2,
// eq. (interp), tensor product).  Pb -= B^T Ub reads Ub[j - 1 + e'] with
// block B[1 - e']^T; Ub -= A^T Pb reads Pb[q + e'] with block A[1 - e']^T.
void build_adjoint_tables(const hl_plan_s* pl, std::vector<double>& tp, std::vector<double>& tu, WeightMode wm) {
  const int d = pl->d, m = pl->m, MP = m + 1, N2 = 2 * m + 2, nc = pl->nc, ne = 1 << d;
  const PolyOps P = poly_ops(pl);
  const std::vector<double> H = hermite_matrix(m);  // [b][L_0..L_m, R_0..R_m]
  const std::vector<double> Wp = weight_operator(pl, P, 1, wm), Wq = weight_operator(pl, P, 0, wm);
  auto row = [&](const int* s) {  // coefficient index of s in {0..2m+1}^d
    int r = 0;
    for (int k = d - 1; k >= 0; --k) r = r * N2 + s[k];
    return r;
  };
  tp.assign((size_t)ne * d * nc * nc, 0.0);
  tu.assign((size_t)ne * d * nc * nc, 0.0);
  std::vector<double> I(P.size);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < nc; ++a) {
      int ad[3] = {0, 0, 0};
      for (int k = 0, r = a; k < d; ++k, r /= MP) ad[k] = r % MP;
      for (int b = 0; b < P.size; ++b) {
        double v = 1.0;
        for (int k = 0; k < d; ++k) v *= H[P.dig(b, k) * N2 + ((e >> k) & 1) * MP + ad[k]];
        I[b] = v;
      }
      const int ep = (ne - 1) ^ e;  // e' = 1 - e
      for (int i = 0; i < d; ++i) {
        const std::vector<double> DI = P.deriv(I, i);
        for (int sidx = 0; sidx < nc; ++sidx) {
          int sd[3] = {0, 0, 0};
          for (int k = 0, r = sidx; k < d; ++k, r /= MP) sd[k] = r % MP;
          const int srow = row(sd);
          double av = 0.0;
          for (int b = 0; b < P.size; ++b) av += Wp[(size_t)srow * P.size + b] * DI[b];
          int se[3] = {sd[0], sd[1], sd[2]};
          se[i] += 1;
          const int serow = row(se);
          double bv = 0.0;
          for (int b = 0; b < P.size; ++b) bv += Wq[(size_t)serow * P.size + b] * I[b];
          bv *= (sd[i] + 1) / pl->h[i];
          // Pb -= B^T Ub: out r = a (1 component), in (ii = i, c = s)
          tp[((((size_t)ep * 1 + 0) * d + i) * nc + a) * nc + sidx] = bv;
          // Ub -= A^T Pb: out (io = i, r = a), in (c = s)
          tu[((((size_t)ep * d + i) * 1 + 0) * nc + a) * nc + sidx] = av;
        }
      }
    }
}

// Build every table of the plan into host FP64 memory (packed as the kernels
// read it, hl_layout.hpp), with the weights of wm.
hl_status build_tables(hl_plan_s* pl, std::vector<double>& tab, WeightMode wm) {
  const int d = pl->d, m = pl->m, MP = m + 1, N2 = 2 * m + 2;
  const hl::KernelSet& ks = pl->ks;
  tab.assign(ks.table_words, 0.0);
  const std::vector<double> H = hermite_matrix(m);  // [s][L.., R..]
  // The kernels rely on the +-1/2 symmetry H[b][L_l] = (-1)^{b+l} H[b][R_l]
  // (sigma/delta form of every pass); check it exactly.
  for (int b = 0; b < N2; ++b)
    for (int l = 0; l < MP; ++l) {
      const double L = H[b * N2 + l], R = H[b * N2 + MP + l];
      const double want = ((b + l) & 1) ? -R : R;
      if (L != want) return fail(HL_ERR_ARG, "internal: interpolation matrix lacks the +-1/2 symmetry");
    }
  // Last-dimension pass coefficient on sigma_l / delta_l: H[b][R_l], or for the
  // derivative pass (b + 1) H[b + 1][R_l] / h_last.
  const int kL = d - 1;
  auto glast = [&](int b, int l, bool dH) -> double {
    if (!dH) return H[b * N2 + MP + l];
    return (b + 1 < N2) ? (b + 1) * H[(b + 1) * N2 + MP + l] / pl->h[kL] : 0.0;
  };

  const PolyOps P = poly_ops(pl);
  int NC = 1, NB = 1;
  for (int k = 0; k < d; ++k) NC *= MP;
  for (int k = 0; k + 1 < d; ++k) NB *= N2;
  const int stride_last = (d == 1) ? 1 : (d == 2 ? N2 : N2 * N2);

  // Output sets: pressure s in {0..m}^d (digits base m+1); velocity: the set
  // G of Q (digits in {0..m+1}, at most one equal to m+1, not all zero).
  std::vector<std::vector<int>> out_p, out_g;
  {
    int total = 1;
    for (int k = 0; k < d; ++k) total *= (m + 2);
    for (int s = 0; s < NC; ++s) {
      std::vector<int> dg(d);
      for (int k = 0, r = s; k < d; ++k, r /= MP) dg[k] = r % MP;
      out_p.push_back(dg);
    }
    for (int x = 0; x < total; ++x) {
      std::vector<int> dg(d);
      int top = 0, nz = 0;
      for (int k = 0, r = x; k < d; ++k, r /= (m + 2)) {
        dg[k] = r % (m + 2);
        top += dg[k] == m + 1;
        nz += dg[k] != 0;
      }
      if (top <= 1 && nz > 0) out_g.push_back(dg);
    }
  }
  if ((int)out_g.size() != ks.ng) return fail(HL_ERR_ARG, "internal: velocity output set size mismatch");

  // Pack a merged table (sigma/delta form):
  //   M[l][o][b] = scale * sum_bL W(o, (b, bL)) glast(bL, l)
  // over the structurally nonzero (o, b); verify the rest is zero and that
  // every contributing bL has the sigma/delta selector the kernel assumes.
  // W(o, beta) = coefficient of xi^o in sum_k c_k Lap^k xi^beta.
  auto pack = [&](const std::vector<double>& W, const std::vector<std::vector<int>>& outs, bool dH_last,
                  double scale, int off) -> hl_status {
    int t = off;
    const int flip = dH_last ? 1 : 0;
    for (int l = 0; l < MP; ++l)
      for (size_t o = 0; o < outs.size(); ++o) {
        const int sel = (outs[o][kL] + l + flip) & 1;
        int orow = 0;  // row of W: o as an index in {0..2m+1}^d
        for (int k = d - 1; k >= 0; --k) orow = orow * N2 + outs[o][k];
        for (int b = 0; b < NB; ++b) {
          double v = 0.0;
          for (int bL = 0; bL < N2; ++bL) {
            const double w = W[(size_t)orow * P.size + b + bL * stride_last];
            if (w == 0.0) continue;
            if (((bL + l + flip) & 1) != sel)
              return fail(HL_ERR_ARG, "internal: merged table mixes sigma and delta terms");
            v += w * glast(bL, l, dH_last);
          }
          v *= scale;
          bool valid = true;
          for (int k = 0; k + 1 < d; ++k) {
            const int bk = (b / (k == 0 ? 1 : N2)) % N2;
            const int r = bk - outs[o][k];
            if (r < 0 || (r & 1)) valid = false;
          }
          if (valid)
            tab[t++] = v;
          else if (v != 0.0)
            return fail(HL_ERR_ARG, "internal: merged table has a nonzero outside its pattern");
        }
      }
    return HL_OK;
  };
  const std::vector<double> Wp = weight_operator(pl, P, 1, wm);   // sum_k w_k kappa^{k+1} Lap^k
  const std::vector<double> Wq = weight_operator(pl, P, 0, wm);   // sum_k w_k kappa^k Lap^k
  hl_status st;
  if (d == 3) {
    // 3D: explicit x pass, y and z merged into the table:
    //   M[a_y, a_z][o][b_x] = scale * sum_{b_y, b_z} W(o, b) gy(b_y, a_y) gz(b_z, a_z)
    // with gy / gz the sigma/delta pass coefficients (derivative pass for the
    // component along that dimension).
    auto gdim = [&](int k, int b, int a, int dH) -> double {
      if (!dH) return H[b * N2 + MP + a];
      return (b + 1 < N2) ? (b + 1) * H[(b + 1) * N2 + MP + a] / pl->h[k] : 0.0;
    };
    int t_end = 0;
    auto pack3 = [&](const std::vector<double>& W, const std::vector<std::vector<int>>& outs, int fy, int fz,
                     double scale, int off) -> hl_status {
      int t = off;
      for (int az = 0; az < MP; ++az)
        for (int ay = 0; ay < MP; ++ay)
          for (size_t o = 0; o < outs.size(); ++o) {
            const int ox = outs[o][0], oy = outs[o][1], oz = outs[o][2];
            const int orow = ox + N2 * (oy + N2 * oz);
            const int ky = (oy + ay + fy) & 1, kz = (oz + az + fz) & 1;
            for (int bx = 0; bx < N2; ++bx) {
              double v = 0.0;
              for (int bz = 0; bz < N2; ++bz)
                for (int by = 0; by < N2; ++by) {
                  const double w = W[(size_t)orow * P.size + bx + N2 * (by + N2 * bz)];
                  if (w == 0.0) continue;
                  if (((by + ay + fy) & 1) != ky || ((bz + az + fz) & 1) != kz)
                    return fail(HL_ERR_ARG, "internal: 3D merged table mixes sigma and delta terms");
                  v += w * gdim(1, by, ay, fy) * gdim(2, bz, az, fz);
                }
              v *= scale;
              if (bx >= ox && ((bx - ox) & 1) == 0)
                tab[t++] = v;
              else if (v != 0.0)
                return fail(HL_ERR_ARG, "internal: 3D merged table has a nonzero outside its pattern");
            }
          }
      t_end = t;
      return HL_OK;
    };
    if ((st = pack3(Wp, out_p, 0, 0, 1.0 / pl->h[0], ks.p_off[0])) != HL_OK) return st;
    if ((st = pack3(Wp, out_p, 1, 0, 1.0, ks.p_off[1])) != HL_OK) return st;
    if ((st = pack3(Wp, out_p, 0, 1, 1.0, ks.p_off[2])) != HL_OK) return st;
    if ((st = pack3(Wq, out_g, 0, 0, 1.0, ks.u_off)) != HL_OK) return st;
    if (ks.f_off >= 0) {
      // fully merged pressure table F[i][a][o] = A[e = upper corner in every
      // dimension][o][i][a] (A: the per-corner operator of the transposed
      // half-steps' construction); every other corner's block must equal it
      // up to the sigma/delta sign (-1 for a lower corner in a dimension whose
      // combination is delta), which the kernel's butterfly assumes
      std::vector<double> tp, tu;
      build_adjoint_tables(pl, tp, tu, wm);
      const int nc = pl->nc;
      // tu[e'][i][a][s] holds A[1 - e'][s][i][a]: e' = 0 is the all-upper corner
      auto Ablk = [&](int e, int i, int s, int a) { return tu[((((size_t)(7 ^ e)) * 3 + i) * nc + a) * nc + s]; };
      int t = ks.f_off;
      for (int i = 0; i < 3; ++i)
        for (int a = 0; a < nc; ++a)
          for (int o = 0; o < nc; ++o) {
            const double F = Ablk(7, i, o, a);
            const int ad[3] = {a % MP, (a / MP) % MP, a / (MP * MP)}, od[3] = {o % MP, (o / MP) % MP, o / (MP * MP)};
            for (int e = 0; e < 8; ++e) {
              double sgn = 1.0;
              for (int k = 0; k < 3; ++k)
                if (!((e >> k) & 1) && ((od[k] + ad[k] + (k == i)) & 1)) sgn = -sgn;
              const double want = sgn * F, got = Ablk(e, i, o, a);
              if (std::fabs(got - want) > 1e-12 * (std::fabs(F) + 1e-300) + 1e-300)
                return fail(HL_ERR_ARG, "internal: fully merged 3D table lacks the sigma/delta symmetry");
            }
            tab[t++] = F;
          }
      t_end = t;
    }
    if (ks.fu_off >= 0) {
      // fully merged velocity table Fu[a][o] = sum_b W_q(o, b) H[b_x][R_ax] H[b_y][R_ay] H[b_z][R_az]
      // (the upper corner's coefficient; the kernel's butterfly gives the
      // others their sign): every contributing b must share the parity of o
      int t = ks.fu_off;
      for (int a = 0; a < pl->nc; ++a) {
        const int ad[3] = {a % MP, (a / MP) % MP, a / (MP * MP)};
        for (size_t o = 0; o < out_g.size(); ++o) {
          const int orow = out_g[o][0] + N2 * (out_g[o][1] + N2 * out_g[o][2]);
          double v = 0.0;
          for (int bz = 0; bz < N2; ++bz)
            for (int by = 0; by < N2; ++by)
              for (int bx = 0; bx < N2; ++bx) {
                const double w = Wq[(size_t)orow * P.size + bx + N2 * (by + N2 * bz)];
                if (w == 0.0) continue;
                const int bd[3] = {bx, by, bz};
                for (int k = 0; k < 3; ++k)
                  if (((bd[k] - out_g[o][k]) & 1) != 0)
                    return fail(HL_ERR_ARG, "internal: fully merged velocity table mixes sigma and delta terms");
                v += w * H[bx * N2 + MP + ad[0]] * H[by * N2 + MP + ad[1]] * H[bz * N2 + MP + ad[2]];
              }
          tab[t++] = v;
        }
      }
      t_end = t;
    }
    if (t_end != ks.table_words) return fail(HL_ERR_ARG, "internal: 3D table size mismatch");
    return HL_OK;
  }
  // x-component (2D): the slice pass gives the x-derivative in units of 1/h_x
  if (d > 1 && (st = pack(Wp, out_p, false, 1.0 / pl->h[0], ks.p_off[0])) != HL_OK) return st;
  if ((st = pack(Wp, out_p, true, 1.0, ks.p_off[d - 1])) != HL_OK) return st;
  if ((st = pack(Wq, out_g, false, 1.0, ks.u_off)) != HL_OK) return st;
  return HL_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

using hl_host::FieldImage;
using hl_host::LayoutMap;

// Field 0 = p (primal), 1 = u (dual).
LayoutMap layout_of(const hl_plan_s* pl, int field) {
  return hl_host::field_layout(pl->d, pl->m, pl->K, pl->walls, field);
}

// field 0: p (one component), field 1: u (d components).
hl_status upload_field(const hl_plan_s* pl, const double* host, int field, void* dev, hipStream_t s) {
  const int ncomp = field == 0 ? 1 : pl->d;
  const LayoutMap L = layout_of(pl, field);
  const int64_t hw = (int64_t)pl->nc * L.K[0] * L.K[1] * L.K[2];  // host words per component
  FieldImage im{pl->precision, (int64_t)pl->nc * L.nodes, {}, {}};
  if (!im.alloc()) return fail(HL_ERR_NOMEM, "hl_init: host staging allocation failed");
  unsigned char* d = static_cast<unsigned char*>(dev);
  for (int i = 0; i < ncomp; ++i) {
    const double* src = host ? host + (size_t)i * hw : nullptr;
    // ghost nodes (walls) start at zero; the library refreshes them before use
    std::fill(im.hi.begin(), im.hi.end(), (unsigned char)0);
    std::fill(im.lo.begin(), im.lo.end(), (unsigned char)0);
    if (src) L.for_each([&](int64_t h, int64_t dv) { im.put(dv, src[h]); });
    hipError_t e = hipMemcpyAsync(d + i * im.hi_bytes(), im.hi.data(), im.hi_bytes(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && im.lo_bytes())
      e = hipMemcpyAsync(d + ncomp * im.hi_bytes() + i * im.lo_bytes(), im.lo.data(), im.lo_bytes(),
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hl_init: copy to device");
  }
  return HL_OK;
}

hl_status download_field(const hl_plan_s* pl, const void* dev, int field, double* host, hipStream_t s) {
  const int ncomp = field == 0 ? 1 : pl->d;
  const LayoutMap L = layout_of(pl, field);
  const int64_t hw = (int64_t)pl->nc * L.K[0] * L.K[1] * L.K[2];
  FieldImage im{pl->precision, (int64_t)pl->nc * L.nodes, {}, {}};
  if (!im.alloc()) return fail(HL_ERR_NOMEM, "hl_export: host staging allocation failed");
  const unsigned char* d = static_cast<const unsigned char*>(dev);
  for (int i = 0; i < ncomp; ++i) {
    hipError_t e = hipMemcpyAsync(im.hi.data(), d + i * im.hi_bytes(), im.hi_bytes(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && im.lo_bytes())
      e = hipMemcpyAsync(im.lo.data(), d + ncomp * im.hi_bytes() + i * im.lo_bytes(), im.lo_bytes(),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hl_export: copy to host");
    double* dst = host + (size_t)i * hw;
    L.for_each([&](int64_t h, int64_t dv) { dst[h] = im.get(dv); });
  }
  return HL_OK;
}

hl::PlanView view(const hl_plan_s* pl) {
  hl::PlanView v;
  v.gp = pl->gp;
  v.gu = pl->gu;
  for (int k = 0; k < 3; ++k) v.uext[k] = pl->uext[k];
  v.tab = pl->dtab;
  v.adj_tab = pl->dadj;
  v.kap_p = pl->dkap_p;
  v.kap_u = pl->dkap_u;
  v.dt = pl->dt;
  v.d = pl->d;
  v.m = pl->m;
  v.precision = pl->precision;
  for (int k = 0; k < 3; ++k) v.ih[k] = 1.0 / pl->h[k];
  return v;
}

hl_status check_plan(const hl_plan_s* pl, const char* who) {
  if (!pl) return fail(HL_ERR_ARG, std::string(who) + ": plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device)
    return fail(HL_ERR_DEVICE, std::string(who) + ": current HIP device differs from the plan's device");
  return HL_OK;
}

// FP64 sum of squares of a state buffer's nodes (ghost nodes excluded);
// grid (kNormBlocks, planes), one partial per (block, plane), summed on the
// host in a fixed order so the result is deterministic.  The counted nodes
// are i + off per dimension, i in [0, K), of an array with extents E.
struct NormBox {
  int32_t K[3], E[3], off;
};

template <class S>
__global__ void sumsq_kernel(typename S::View v, NormBox b, double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t count = (int64_t)b.K[0] * b.K[1] * b.K[2];
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < count; n += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i0 = n % b.K[0], r = n / b.K[0];
    const int64_t i1 = r % b.K[1], i2 = r / b.K[1];
    const int64_t o1 = b.K[1] > 1 || b.E[1] > 1 ? b.off : 0, o2 = b.K[2] > 1 || b.E[2] > 1 ? b.off : 0;
    const uint32_t node = (uint32_t)((i0 + b.off) + (int64_t)b.E[0] * ((i1 + o1) + (int64_t)b.E[1] * (i2 + o2)));
    const double x = (double)S::load(v, (int)blockIdx.y, node);
    acc = fma(x, x, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

template <class S>
hl_status sumsq_as(const hl_plan_s* pl, const void* x, int field, double* out) {
  const int ncomp = field == 0 ? 1 : pl->d;
  const int planes = ncomp * pl->nc;
  const LayoutMap L = layout_of(pl, field);
  NormBox b;
  for (int k = 0; k < 3; ++k) {
    b.K[k] = (int32_t)L.K[k];
    b.E[k] = (int32_t)L.E[k];
  }
  b.off = (int32_t)L.off;
  const typename S::View v = S::make(x, ncomp, pl->nc, L.nodes);
  hipLaunchKernelGGL(sumsq_kernel<S>, dim3(kNormBlocks, (unsigned)planes), dim3(256), 0, 0, v, b, pl->dpartial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "hl_norms: launch");
  std::vector<double> part((size_t)kNormBlocks * planes);
  e = hipMemcpy(part.data(), pl->dpartial, part.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hl_norms: copy");
  double acc = 0.0;
  for (double t : part) acc += t;
  *out = acc;
  return HL_OK;
}

hl_status sumsq(const hl_plan_s* pl, const void* x, int field, double* out) {
  switch (pl->precision) {
    case HL_FP64: return sumsq_as<hl::PlainStore<double>>(pl, x, field, out);
    case HL_FP32: return sumsq_as<hl::PlainStore<float>>(pl, x, field, out);
    default: return sumsq_as<hl::SplitStore>(pl, x, field, out);
  }
}

// <a, b> over `planes` coefficient planes of `nodes` entries (periodic state
// buffers: every entry counts), FP64 accumulation; one partial per block.
template <class S>
__global__ void dot_kernel(typename S::View a, typename S::View b, int planes, double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int pl = 0; pl < planes; ++pl)
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.nodes; n += (int64_t)gridDim.x * blockDim.x)
      acc = fma((double)S::load(a, pl, (uint32_t)n), (double)S::load(b, pl, (uint32_t)n), acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// *acc += sum of n partials, in a fixed order (one block of 256).
__global__ void add_partials(const double* __restrict__ partial, int n, double* __restrict__ acc) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += partial[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

// *acc += <a, b> for two p-shaped (field 0) or u-shaped (field 1) buffers.
// Bytes per stored coefficient (FP32_COMP: an FP32 hi word and a BF16 lo word).
size_t state_bytes(const hl_plan_s* pl) { return (size_t)pl->word_bytes * pl->words_per_coef; }

hipError_t dot_into(const hl_plan_s* pl, const void* a, const void* b, int field, double* acc, hipStream_t s) {
  const int planes = (field == 0 ? 1 : pl->d) * pl->nc;
  const int64_t nodes = field == 0 ? pl->pnodes : pl->unodes;
  const int ncomp = field == 0 ? 1 : pl->d;
  if (pl->precision == HL_FP64) {
    using S = hl::PlainStore<double>;
    hipLaunchKernelGGL(dot_kernel<S>, dim3(kNormBlocks), dim3(256), 0, s, S::make(a, ncomp, pl->nc, nodes),
                       S::make(b, ncomp, pl->nc, nodes), planes, pl->gpart);
  } else if (pl->precision == HL_FP32_COMP) {
    using S = hl::SplitStore;
    hipLaunchKernelGGL(dot_kernel<S>, dim3(kNormBlocks), dim3(256), 0, s, S::make(a, ncomp, pl->nc, nodes),
                       S::make(b, ncomp, pl->nc, nodes), planes, pl->gpart);
  } else {
    using S = hl::PlainStore<float>;
    hipLaunchKernelGGL(dot_kernel<S>, dim3(kNormBlocks), dim3(256), 0, s, S::make(a, ncomp, pl->nc, nodes),
                       S::make(b, ncomp, pl->nc, nodes), planes, pl->gpart);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(add_partials, dim3(1), dim3(256), 0, s, (const double*)pl->gpart, kNormBlocks, acc);
  return hipGetLastError();
}

// p += a g over every stored coefficient of a p-shaped buffer.
template <class S>
__global__ void axpy_kernel(typename S::View p, typename S::View g, int planes, double a) {
  using T = typename S::C;
  const T at = (T)a;
  for (int pl = 0; pl < planes; ++pl)
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.nodes; n += (int64_t)gridDim.x * blockDim.x) {
      const T gv = S::load(g, pl, (uint32_t)n);
      S::update(p, pl, (uint32_t)n, [&](T x) { return fma(at, gv, x); });
    }
}

hipError_t upload_table(const hl_plan_s* pl, const std::vector<double>& tab, void** out) {
  const size_t bytes = std::max<size_t>(tab.size() * pl->tab_bytes, 16);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return e;
  if (pl->tab_bytes == 8) return hipMemcpy(*out, tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
  std::vector<float> f(tab.begin(), tab.end());
  return hipMemcpy(*out, f.data(), f.size() * 4, hipMemcpyHostToDevice);
}

// Gradient resources of a periodic plan (first use only).
hl_status ensure_gradient(hl_plan_s* pl) {
  if (pl->tab_dk) return HL_OK;
  std::vector<double> tdk, trev;
  hl_status st = build_tables(pl, tdk, WeightMode{pl->dt, true});
  if (st == HL_OK) st = build_tables(pl, trev, WeightMode{-pl->dt, false});
  if (st != HL_OK) return st;
  const size_t pbytes = (size_t)pl->nc * pl->pnodes * state_bytes(pl);
  const size_t ubytes = (size_t)pl->d * pl->nc * pl->unodes * state_bytes(pl);
  hipError_t e = upload_table(pl, tdk, &pl->tab_dk);
  if (e == hipSuccess) e = upload_table(pl, trev, &pl->tab_rev);
  if (e == hipSuccess) e = hipMalloc(&pl->fp, pbytes);
  if (e == hipSuccess) e = hipMalloc(&pl->fu, ubytes);
  if (e == hipSuccess) e = hipMalloc(&pl->sp, pbytes);
  if (e == hipSuccess) e = hipMalloc(&pl->su, ubytes);
  if (e == hipSuccess) e = hipMalloc((void**)&pl->gpart, kNormBlocks * sizeof(double));
  if (e != hipSuccess) {
    for (void** q : {&pl->tab_dk, &pl->tab_rev, &pl->fp, &pl->fu, &pl->sp, &pl->su, (void**)&pl->gpart}) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
    }
    return fail(HL_ERR_NOMEM, std::string("hl_adjoint_step: gradient buffers: ") + hipGetErrorString(e));
  }
  return HL_OK;
}

int64_t kappa_planes(const hl_plan_s* pl) {
  int64_t n = 1;
  for (int k = 0; k < pl->d; ++k) n *= 2 * pl->m + 2;
  return n;
}

hl_status ensure_var_gradient(hl_plan_s* pl) {
  if (pl->gkp) return HL_OK;
  const int64_t np = kappa_planes(pl);
  const size_t gp = (size_t)np * pl->pnodes * sizeof(double), gu = (size_t)np * pl->unodes * sizeof(double);
  const size_t sc = (size_t)pl->d * np * std::max(pl->pnodes, pl->unodes) * pl->tab_bytes;
  hipError_t e = hipMalloc((void**)&pl->gkp, gp);
  if (e == hipSuccess) e = hipMalloc((void**)&pl->gku, gu);
  if (e == hipSuccess) e = hipMalloc(&pl->vscr, sc);
  if (e == hipSuccess) e = hipMemset(pl->gkp, 0, gp);
  if (e == hipSuccess) e = hipMemset(pl->gku, 0, gu);
  if (e != hipSuccess) {
    for (void** q : {(void**)&pl->gkp, (void**)&pl->gku, &pl->vscr}) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
    }
    return fail(HL_ERR_NOMEM, std::string("hl_adjoint_step_var: gradient buffers: ") + hipGetErrorString(e));
  }
  return HL_OK;
}

// Launch grid of one half-step: updates K[] nodes stored at index j + ooff
// of an array with extents oext, corners from an array with extents sext
// (lower corner at j + soff).
bool make_grid(const hl_plan_s* pl, const int32_t* tile, int32_t ygroup, const int32_t* K, const int32_t* oext,
               int32_t ooff, const int32_t* sext, int32_t soff, int64_t onodes, int64_t snodes, hl::Grid* g) {
  int64_t tiles = 1;
  for (int k = 0; k < 3; ++k) {
    g->K[k] = K[k];
    g->nt[k] = (K[k] + tile[k] - 1) / tile[k];
    g->oext[k] = oext[k];
    g->sext[k] = sext[k];
    tiles *= g->nt[k];
  }
  if (tiles > (int64_t)INT32_MAX / 2) return false;
  g->tiles = (int32_t)tiles;
  g->per_xcd = (int32_t)((tiles + hl::kXcds - 1) / hl::kXcds);
  // 3D: tile numbering x, then y in groups of `ygroup` tile rows, then z
  // (z-neighbour planes reused from L2); 1D/2D: plain row-major
  g->ygroup = pl->d == 3 ? std::max<int32_t>(1, std::min<int32_t>(ygroup, g->nt[1])) : g->nt[1];
  g->ooff = ooff;
  g->soff = soff;
  g->tx = tile[0];
  g->ty = tile[1];
  g->pad = 0;
  g->onodes = onodes;
  g->snodes = snodes;
  return true;
}

// The two half-step grids of a plan for a tile shape (tx, ty) and 3D y-group:
// p half-step: primal nodes (walls: K+1, on the walls too) from dual corners
// q = j - 1 + e, stored at q + uoff; u half-step: dual nodes from primal
// corners j = q + e.
bool build_grids(const hl_plan_s* pl, int32_t tx, int32_t ty, int32_t ygroup, hl::Grid* gp, hl::Grid* gu) {
  int32_t Kp[3], Ku[3];
  for (int k = 0; k < 3; ++k) {
    Kp[k] = pl->pext[k];
    Ku[k] = pl->K[k];
  }
  const int32_t tile[3] = {tx, ty, 1};
  return make_grid(pl, tile, ygroup, Kp, pl->pext, 0, pl->uext, pl->uoff - 1, pl->pnodes, pl->unodes, gp) &&
         make_grid(pl, tile, ygroup, Ku, pl->uext, pl->uoff, pl->pext, 0, pl->unodes, pl->pnodes, gu);
}

// Tile shapes a plan may use: x extent a multiple of 32 (whole or half
// wavefronts along the coalesced axis), 64..256 work-items.
bool valid_tile(int d, int32_t tx, int32_t ty) {
  if (tx < 32 || tx > 256 || tx % 32 != 0 || ty < 1) return false;
  if (d == 1 && ty != 1) return false;
  const int32_t n = tx * ty;
  return n >= 64 && n <= 256;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// hl_norms_noalloc: hl_norms with its block partials in a file-scope device
// array instead of the plan's buffer, for callers that cannot allocate.  Host
// code never passes `norm_scratch` itself to a kernel (in host code the name
// is a stand-in, not a device address): each device's address comes from
// hipGetSymbolAddress, taken once per device on the first call there.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoAllocMaxPlanes = 3 * 64;  // d nc for 3D m = 3, the largest built
constexpr size_t kNoAllocWords = (size_t)kNormBlocks * kNoAllocMaxPlanes + 2;
static __device__ __align__(256) double norm_scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_of_device(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(norm_scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// out[0] = sum of the first n partials, in a fixed order (one block of 256).
__global__ void sum_partials(const double* __restrict__ partial, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += partial[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <class S>
hipError_t sumsq_static(const hl_plan_s* pl, const void* x, int field, double* scr, double* res) {
  const int ncomp = field == 0 ? 1 : pl->d;
  const int planes = ncomp * pl->nc;
  const LayoutMap L = layout_of(pl, field);
  NormBox b;
  for (int k = 0; k < 3; ++k) {
    b.K[k] = (int32_t)L.K[k];
    b.E[k] = (int32_t)L.E[k];
  }
  b.off = (int32_t)L.off;
  const typename S::View v = S::make(x, ncomp, pl->nc, L.nodes);
  hipLaunchKernelGGL(sumsq_kernel<S>, dim3(kNormBlocks, (unsigned)planes), dim3(256), 0, 0, v, b, scr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, 0, (const double*)scr, kNormBlocks * planes, res);
  return hipGetLastError();
}

hipError_t sumsq_static_any(const hl_plan_s* pl, const void* x, int field, double* scr, double* res) {
  switch (pl->precision) {
    case HL_FP64: return sumsq_static<hl::PlainStore<double>>(pl, x, field, scr, res);
    case HL_FP32: return sumsq_static<hl::PlainStore<float>>(pl, x, field, scr, res);
    default: return sumsq_static<hl::SplitStore>(pl, x, field, scr, res);
  }
}

}  // namespace

extern "C" {

const char* hl_last_error(void) { return g_last_error.c_str(); }

hl_status hl_plan(const hl_problem* prob, hl_plan_t* out) {
  g_last_error.clear();
  if (!prob || !out) return fail(HL_ERR_ARG, "hl_plan: NULL argument");
  const hl_problem& p = *prob;
  if (p.reserved[0] != 0 || p.reserved[1] != 0) return fail(HL_ERR_ARG, "hl_plan: reserved fields must be 0");
  if (p.boundary != HL_PERIODIC && p.boundary != HL_WALLS) return fail(HL_ERR_ARG, "hl_plan: unknown boundary");
  if (p.d < 1 || p.d > 3) return fail(HL_ERR_ARG, "hl_plan: d must be 1, 2 or 3");
  if (p.m < 0) return fail(HL_ERR_ARG, "hl_plan: m must be >= 0");
  if (p.m > max_m(p.d)) return fail(HL_ERR_UNSUPPORTED, "hl_plan: m too large for this dimension");
  if (p.precision != HL_FP64 && p.precision != HL_FP32 && p.precision != HL_FP32_COMP)
    return fail(HL_ERR_ARG, "hl_plan: unknown precision");
  if (!finite_pos(p.c)) return fail(HL_ERR_ARG, "hl_plan: c must be finite and > 0");
  double hmin = INFINITY;
  int64_t max_nodes = 1;  // largest device array (walls: the ghost-padded velocity)
  for (int k = 0; k < p.d; ++k) {
    if (p.cells[k] < 2 || p.cells[k] > (int64_t)INT32_MAX - 2) return fail(HL_ERR_ARG, "hl_plan: cells must be in [2, 2^31 - 2)");
    if (!finite_pos(p.length[k])) return fail(HL_ERR_ARG, "hl_plan: length must be finite and > 0");
    hmin = std::min(hmin, p.length[k] / (double)p.cells[k]);
    max_nodes *= p.cells[k] + (p.boundary == HL_WALLS ? 2 : 0);
  }
  double dt = p.dt;
  if (!std::isfinite(dt) || dt < 0.0) return fail(HL_ERR_ARG, "hl_plan: dt must be finite and >= 0");
  if (dt == 0.0) {
    if (!std::isfinite(p.cfl) || !(p.cfl > 0.0 && p.cfl < 1.0))
      return fail(HL_ERR_CFL, "hl_plan: cfl must be in (0, 1) when dt == 0");
    dt = p.cfl * hmin / p.c;
  }
  const double nu = p.c * dt / hmin;
  if (!(nu > 0.0 && nu < 1.0)) return fail(HL_ERR_CFL, "hl_plan: c dt / min h must be in (0, 1)");

  hl_plan_s* pl = new (std::nothrow) hl_plan_s();
  if (!pl) return fail(HL_ERR_NOMEM, "hl_plan: out of host memory");
  pl->prob = p;
  pl->d = p.d;
  pl->m = p.m;
  pl->precision = p.precision;
  pl->word_bytes = p.precision == HL_FP64 ? 8 : (p.precision == HL_FP32 ? 4 : 2);
  pl->words_per_coef = p.precision == HL_FP32_COMP ? 3 : 1;
  pl->tab_bytes = p.precision == HL_FP32 ? 4 : 8;
  pl->dt = dt;
  pl->nu = nu;
  pl->kappa = p.c * p.c;
  pl->nc = 1;
  for (int k = 0; k < p.d; ++k) pl->nc *= (p.m + 1);
  pl->walls = p.boundary == HL_WALLS;
  pl->uoff = pl->walls ? 1 : 0;
  for (int k = 0; k < 3; ++k) {
    pl->h[k] = k < p.d ? p.length[k] / (double)p.cells[k] : 1.0;
    pl->K[k] = k < p.d ? (int32_t)p.cells[k] : 1;
  }
  {
    const LayoutMap lp = layout_of(pl, 0), lu = layout_of(pl, 1);
    for (int k = 0; k < 3; ++k) {
      pl->pext[k] = (int32_t)lp.E[k];
      pl->uext[k] = (int32_t)lu.E[k];
    }
    pl->pnodes = lp.nodes;
    pl->unodes = lu.nodes;
  }
  // the widest plane: FP64 words, or the FP32 (hi) planes
  if ((double)max_nodes * (p.precision == HL_FP64 ? 8 : 4) >= 4294967296.0) {
    delete pl;
    return fail(HL_ERR_UNSUPPORTED, "hl_plan: one coefficient plane must stay below 4 GiB");
  }
  const bool ok = hl::kernels_for(p.d, p.m, p.precision, &pl->ks);
  if (!ok) {
    delete pl;
    return fail(HL_ERR_UNSUPPORTED, "hl_plan: (d, m, precision) not built");
  }
  pl->ygroup_req = kYGroup3;
  if (!build_grids(pl, pl->ks.tile[0], pl->ks.tile[1], kYGroup3, &pl->gp, &pl->gu)) {
    delete pl;
    return fail(HL_ERR_UNSUPPORTED, "hl_plan: grid too large for the launch");
  }
  std::vector<double> tab;
  hl_status st = build_tables(pl, tab, WeightMode{pl->dt, false});
  if (st != HL_OK) {
    delete pl;
    return st;
  }
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    delete pl;
    return hip_fail(e, "hl_plan: hipGetDevice");
  }
  const size_t bytes = tab.size() * pl->tab_bytes;
  e = hipMalloc(&pl->dtab, std::max<size_t>(bytes, 16));
  if (e == hipSuccess) e = hipMalloc((void**)&pl->dpartial, (size_t)kNormBlocks * pl->d * pl->nc * sizeof(double));
  if (e != hipSuccess) {
    if (pl->dtab) (void)hipFree(pl->dtab);
    delete pl;
    return fail(HL_ERR_NOMEM, std::string("hl_plan: device allocation: ") + hipGetErrorString(e));
  }
  if (pl->tab_bytes == 8) {
    e = hipMemcpy(pl->dtab, tab.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> tf(tab.begin(), tab.end());
    e = hipMemcpy(pl->dtab, tf.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipFree(pl->dtab);
    (void)hipFree(pl->dpartial);
    delete pl;
    return hip_fail(e, "hl_plan: table upload");
  }
  if (pl->ks.adj_p) {
    std::vector<double> tp, tu;
    build_adjoint_tables(pl, tp, tu, WeightMode{pl->dt, false});
    pl->adj_u_off = tp.size();
    const size_t n = tp.size() + tu.size();
    e = hipMalloc(&pl->dadj, n * pl->tab_bytes);
    if (e == hipSuccess) {
      std::vector<double> all(tp);
      all.insert(all.end(), tu.begin(), tu.end());
      if (pl->tab_bytes == 8) {
        e = hipMemcpy(pl->dadj, all.data(), n * 8, hipMemcpyHostToDevice);
      } else {
        std::vector<float> f(all.begin(), all.end());
        e = hipMemcpy(pl->dadj, f.data(), n * 4, hipMemcpyHostToDevice);
      }
    }
    if (e != hipSuccess) {
      if (pl->dadj) (void)hipFree(pl->dadj);
      (void)hipFree(pl->dtab);
      (void)hipFree(pl->dpartial);
      delete pl;
      return hip_fail(e, "hl_plan: adjoint table upload");
    }
  }
  *out = pl;
  return HL_OK;
}

hl_status hl_plan_destroy(hl_plan_t plan) {
  g_last_error.clear();
  if (!plan) return HL_OK;
  drop_graph(plan);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  if (plan->dtab) (void)hipFree(plan->dtab);
  if (plan->dadj) (void)hipFree(plan->dadj);
  for (void* q : {plan->dkap_p, plan->dkap_u, plan->tab_dk, plan->tab_rev, plan->fp, plan->fu, plan->sp, plan->su,
                  (void*)plan->gpart, (void*)plan->gkp, (void*)plan->gku, plan->vscr, plan->wscr, plan->vzw,
                  plan->ucw})
    if (q) (void)hipFree(q);
  if (plan->dpartial) (void)hipFree(plan->dpartial);
  delete plan;
  return HL_OK;
}

hl_status hl_plan_info(hl_plan_t plan, hl_info* out) {
  g_last_error.clear();
  if (!plan || !out) return fail(HL_ERR_ARG, "hl_plan_info: NULL argument");
  out->dt = plan->dt;
  out->nu = plan->nu;
  out->nodes = plan->pnodes;
  out->nc = plan->nc;
  out->word_bytes = plan->word_bytes;
  out->p_words = (int64_t)plan->words_per_coef * plan->nc * plan->pnodes;
  out->tile[0] = plan->gp.tx;
  out->tile[1] = plan->gp.ty;
  out->ygroup = plan->d == 3 ? plan->gp.ygroup : 0;
  out->reserved = 0;
  out->u_words = (int64_t)plan->words_per_coef * plan->d * plan->nc * plan->unodes;
  return HL_OK;
}

hl_status hl_init(hl_plan_t plan, const double* p0, const double* u0, uint32_t flags, void* p, void* u,
                  void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_init");
  if (st != HL_OK) return st;
  if (!p0 || !p) return fail(HL_ERR_ARG, "hl_init: p0 and p must be non-NULL");
  if (flags & ~HL_INIT_STARTUP) return fail(HL_ERR_ARG, "hl_init: unknown flags");
  if (!u && (u0 || (flags & HL_INIT_STARTUP)))
    return fail(HL_ERR_ARG, "hl_init: u may be NULL only without u0 and without the start-up");
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_field(plan, p0, 0, p, s)) != HL_OK) return st;
  if (u && (st = upload_field(plan, u0, 1, u, s)) != HL_OK) return st;
  if (flags & HL_INIT_STARTUP) {
    hipError_t e = u_fn(plan)(view(plan), u, p, 0.5, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hl_init: start-up half-step");
  }
  return HL_OK;
}

hl_status hl_export(hl_plan_t plan, const void* p, const void* u, double* p_out, double* u_out, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_export");
  if (st != HL_OK) return st;
  if ((p_out && !p) || (u_out && !u)) return fail(HL_ERR_ARG, "hl_export: NULL device buffer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hl_export: pending work failed");
  if (p_out && (st = download_field(plan, p, 0, p_out, s)) != HL_OK) return st;
  if (u_out && (st = download_field(plan, u, 1, u_out, s)) != HL_OK) return st;
  return HL_OK;
}

hl_status hl_p_half(hl_plan_t plan, void* p, void* u, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_p_half");
  if (st != HL_OK) return st;
  if (!p || !u || p == u) return fail(HL_ERR_ARG, "hl_p_half: p and u must be distinct non-NULL buffers");
  const hl::PlanView v = view(plan);
  hipError_t e = plan->walls ? plan->ks.ghost(v, u, (hipStream_t)stream) : hipSuccess;
  if (e == hipSuccess) e = p_fn(plan)(v, p, u, (hipStream_t)stream);
  return e == hipSuccess ? HL_OK : hip_fail(e, "hl_p_half: launch");
}

hl_status hl_u_half(hl_plan_t plan, void* u, const void* p, double weight_scale, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_u_half");
  if (st != HL_OK) return st;
  if (!p || !u || p == u) return fail(HL_ERR_ARG, "hl_u_half: p and u must be distinct non-NULL buffers");
  if (!std::isfinite(weight_scale)) return fail(HL_ERR_ARG, "hl_u_half: weight_scale must be finite");
  hipError_t e = u_fn(plan)(view(plan), u, p, weight_scale, (hipStream_t)stream);
  return e == hipSuccess ? HL_OK : hip_fail(e, "hl_u_half: launch");
}

hl_status hl_step(hl_plan_t plan, void* p, void* u, int64_t nsteps, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_step");
  if (st != HL_OK) return st;
  if (!p || !u || p == u) return fail(HL_ERR_ARG, "hl_step: p and u must be distinct non-NULL buffers");
  if (nsteps < 0) return fail(HL_ERR_ARG, "hl_step: nsteps must be >= 0");
  const hl::PlanView v = view(plan);
  hipStream_t s = (hipStream_t)stream;
  int64_t n = 0;
  if (nsteps >= kGraphChunk) {
    if (!plan->gexec || plan->graph_p != p || plan->graph_u != u) {
      hipError_t e = capture_steps(plan, v, p, u);
      if (e != hipSuccess) return hip_fail(e, "hl_step: graph capture");
    }
    for (; n + kGraphChunk <= nsteps; n += kGraphChunk) {
      hipError_t e = hipGraphLaunch(plan->gexec, s);
      if (e != hipSuccess) return hip_fail(e, "hl_step: graph launch");
    }
  }
  for (; n < nsteps; ++n) {
    hipError_t e = plan->walls ? plan->ks.ghost(v, u, s) : hipSuccess;
    if (e == hipSuccess) e = p_fn(plan)(v, p, u, s);
    if (e == hipSuccess) e = u_fn(plan)(v, u, p, 1.0, s);
    if (e != hipSuccess) return hip_fail(e, "hl_step: launch");
  }
  return HL_OK;
}

hl_status hl_add_source(hl_plan_t plan, void* p, const void* g, double a, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_add_source");
  if (st != HL_OK) return st;
  if (!p || !g || p == g) return fail(HL_ERR_ARG, "hl_add_source: p and g must be distinct non-NULL buffers");
  if (!std::isfinite(a)) return fail(HL_ERR_ARG, "hl_add_source: a must be finite");
  hipStream_t s = (hipStream_t)stream;
  const int planes = plan->nc;
  const int64_t nodes = plan->pnodes;
  const unsigned blocks = (unsigned)std::min<int64_t>(2048, (nodes + 255) / 256);
  switch (plan->precision) {
    case HL_FP64: {
      using S = hl::PlainStore<double>;
      hipLaunchKernelGGL(axpy_kernel<S>, dim3(blocks), dim3(256), 0, s, S::make(p, 1, planes, nodes),
                         S::make(g, 1, planes, nodes), planes, a);
      break;
    }
    case HL_FP32: {
      using S = hl::PlainStore<float>;
      hipLaunchKernelGGL(axpy_kernel<S>, dim3(blocks), dim3(256), 0, s, S::make(p, 1, planes, nodes),
                         S::make(g, 1, planes, nodes), planes, a);
      break;
    }
    default: {
      using S = hl::SplitStore;
      hipLaunchKernelGGL(axpy_kernel<S>, dim3(blocks), dim3(256), 0, s, S::make(p, 1, planes, nodes),
                         S::make(g, 1, planes, nodes), planes, a);
    }
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HL_OK : hip_fail(e, "hl_add_source: launch");
}

hl_status hl_set_kappa(hl_plan_t plan, const double* kappa_p, const double* kappa_u) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_set_kappa");
  if (st != HL_OK) return st;
  if (!kappa_p != !kappa_u) return fail(HL_ERR_ARG, "hl_set_kappa: give both kappa arrays or neither");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hl_set_kappa: pending work failed");
  drop_graph(plan);
  ++plan->gen;
  if (!kappa_p) {  // back to the constant kappa of the plan
    plan->var_kappa = false;
    for (void** q : {&plan->dkap_p, &plan->dkap_u}) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
    }
    return HL_OK;
  }
  if (!plan->ks.p_half_var) return fail(HL_ERR_UNSUPPORTED, "hl_set_kappa: variable kappa is not built for this plan");
  // host layout [nodes][b_1..b_d], b_k in 0..2m+1: the field layout of order
  // 2m+1 of p (primal nodes, K+1 per dimension with walls) and of one velocity
  // component (dual nodes; with walls stored in the padded array, whose ghost
  // entries the kernels never read)
  const double* srcs[2] = {kappa_p, kappa_u};
  void** dsts[2] = {&plan->dkap_p, &plan->dkap_u};
  for (int f = 0; f < 2; ++f) {
    const LayoutMap L = hl_host::field_layout(plan->d, 2 * plan->m + 1, plan->K, plan->walls, f);
    const int64_t hw = (int64_t)L.nc * L.K[0] * L.K[1] * L.K[2];
    for (int64_t i = 0; i < hw; ++i)
      if (!std::isfinite(srcs[f][i])) return fail(HL_ERR_ARG, "hl_set_kappa: kappa data must be finite");
  }
  for (int f = 0; f < 2; ++f) {
    const LayoutMap L = hl_host::field_layout(plan->d, 2 * plan->m + 1, plan->K, plan->walls, f);
    FieldImage im{plan->precision, (int64_t)L.nc * L.nodes, {}, {}};
    if (!im.alloc()) return fail(HL_ERR_NOMEM, "hl_set_kappa: host staging allocation failed");
    // the kappa data in the plan's storage (FP32_COMP: hi planes, then lo planes)
    if (!*dsts[f] && (e = hipMalloc(dsts[f], im.hi_bytes() + im.lo_bytes())) != hipSuccess)
      return fail(HL_ERR_NOMEM, std::string("hl_set_kappa: device allocation: ") + hipGetErrorString(e));
    L.for_each([&](int64_t h, int64_t dv) { im.put(dv, srcs[f][h]); });
    e = hipMemcpy(*dsts[f], im.hi.data(), im.hi_bytes(), hipMemcpyHostToDevice);
    if (e == hipSuccess && im.lo_bytes())
      e = hipMemcpy(static_cast<char*>(*dsts[f]) + im.hi_bytes(), im.lo.data(), im.lo_bytes(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hl_set_kappa: copy to device");
  }
  plan->var_kappa = true;
  return HL_OK;
}

hl_status hl_norms(hl_plan_t plan, const void* p, const void* u, double* out) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_norms");
  if (st != HL_OK) return st;
  if (!p || !u || !out) return fail(HL_ERR_ARG, "hl_norms: NULL argument");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hl_norms: pending work failed");
  if ((st = sumsq(plan, p, 0, &out[0])) != HL_OK) return st;
  if ((st = sumsq(plan, u, 1, &out[1])) != HL_OK) return st;
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(HL_ERR_NONFINITE, "hl_norms: non-finite state");
  return HL_OK;
}

hl_status hl_norms_noalloc(hl_plan_t plan, const void* p, const void* u, double* out) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_norms_noalloc");
  if (st != HL_OK) return st;
  if (!p || !u || !out) return fail(HL_ERR_ARG, "hl_norms_noalloc: NULL argument");
  if (plan->d * plan->nc > kNoAllocMaxPlanes)
    return fail(HL_ERR_UNSUPPORTED, "hl_norms_noalloc: more coefficient planes than its scratch holds");
  double* scr = nullptr;
  hipError_t e = scratch_of_device(plan->device, &scr);
  if (e != hipSuccess) return hip_fail(e, "hl_norms_noalloc: scratch address");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hl_norms_noalloc: pending work failed");
  // partials in scr[0, kNormBlocks * planes); the two sums in the last two words
  double* res = scr + (kNoAllocWords - 2);
  e = sumsq_static_any(plan, p, 0, scr, res);
  if (e == hipSuccess) e = sumsq_static_any(plan, u, 1, scr, res + 1);
  if (e == hipSuccess) e = hipMemcpy(out, res, 2 * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hl_norms_noalloc: launch or copy");
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return fail(HL_ERR_NONFINITE, "hl_norms_noalloc: non-finite state");
  return HL_OK;
}

hl_status hl_adjoint_step(hl_plan_t plan, void* p_bar, void* u_bar, const void* p, const void* u,
                          void* grad_kappa, int64_t nsteps, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_adjoint_step");
  if (st != HL_OK) return st;
  if (plan->var_kappa) return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step: built for constant kappa only");
  if (grad_kappa && (!p || !u)) return fail(HL_ERR_ARG, "hl_adjoint_step: the gradient needs the forward state p, u");
  if (!plan->dadj) return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step: not built for this (d, m, precision)");
  if (!p_bar || !u_bar || p_bar == u_bar)
    return fail(HL_ERR_ARG, "hl_adjoint_step: p_bar and u_bar must be distinct non-NULL buffers");
  if (nsteps < 0) return fail(HL_ERR_ARG, "hl_adjoint_step: nsteps must be >= 0");
  hl::PlanView v = view(plan);
  hipStream_t s = (hipStream_t)stream;
  const char* tab = static_cast<const char*>(plan->dadj);
  hl::PlanView vb = v, va = v;
  vb.adj_tab = tab;                                            // B^T blocks
  va.adj_tab = tab + plan->adj_u_off * (size_t)plan->tab_bytes;  // A^T blocks
  if (plan->walls) {
    // A^T on the whole padded velocity array (K + 2 slots per dimension),
    // primal corners j = r - 1 + e from the K + 1 primal nodes
    hl::Grid gf;
    const int32_t tile[3] = {plan->gu.tx, plan->gu.ty, 1};
    if (!make_grid(plan, tile, plan->gu.ygroup, plan->uext, plan->uext, 0, plan->pext, -1, plan->unodes,
                   plan->pnodes, &gf))
      return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step: grid too large for the launch");
    if (!plan->wscr) {
      const size_t ub = (size_t)plan->d * plan->nc * plan->unodes * state_bytes(plan);
      hipError_t e = hipMalloc(&plan->wscr, ub);
      if (e == hipSuccess) e = hipMemset(plan->wscr, 0, ub);  // the fold leaves it zeroed after each use
      if (e != hipSuccess) {
        if (plan->wscr) (void)hipFree(plan->wscr);
        plan->wscr = nullptr;
        return fail(HL_ERR_NOMEM, std::string("hl_adjoint_step: wall scratch: ") + hipGetErrorString(e));
      }
    }
    hipError_t e = plan->ks.ghost_zero(v, u_bar, s);
    if (!grad_kappa) {
      for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
        e = plan->ks.adj_p(vb, p_bar, u_bar, s);                              // Pb -= B^T Ub
        if (e == hipSuccess) e = plan->ks.adj_u_walls(va, gf, u_bar, p_bar, plan->wscr, s);  // Ub -= G^T A^T Pb
      }
      return e == hipSuccess ? HL_OK : hip_fail(e, "hl_adjoint_step: launch");
    }
    // the periodic gradient's walk (below), with A G in place of A: the ghost
    // refresh of U_t before the pressure-side operators read it
    if ((st = ensure_gradient(plan)) != HL_OK) return st;
    hl::PlanView vdk = v, vrev = v;
    vdk.tab = plan->tab_dk;
    vrev.tab = plan->tab_rev;
    const size_t pbytes = (size_t)plan->nc * plan->pnodes * state_bytes(plan);
    const size_t ubytes = (size_t)plan->d * plan->nc * plan->unodes * state_bytes(plan);
    double* g = static_cast<double*>(grad_kappa);
    if (e == hipSuccess) e = hipMemcpyAsync(plan->fp, p, pbytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(plan->fu, u, ubytes, hipMemcpyDeviceToDevice, s);
    for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
      e = hipMemsetAsync(plan->su, 0, ubytes, s);
      if (e == hipSuccess) e = plan->ks.u_half(vdk, plan->su, plan->fp, 1.0, s);       // su = -B_kappa P'
      if (e == hipSuccess) e = dot_into(plan, u_bar, plan->su, 1, g, s);
      if (e == hipSuccess) e = plan->ks.u_half(v, plan->fu, plan->fp, -1.0, s);       // fu = U_t
      if (e == hipSuccess) e = plan->ks.adj_p(vb, p_bar, u_bar, s);                    // Pb -= B^T Ub
      if (e == hipSuccess) e = plan->ks.ghost(v, plan->fu, s);                         // G U_t
      if (e == hipSuccess) e = hipMemsetAsync(plan->sp, 0, pbytes, s);
      if (e == hipSuccess) e = plan->ks.p_half(vdk, plan->sp, plan->fu, s);             // sp = -A_kappa G U_t
      if (e == hipSuccess) e = dot_into(plan, p_bar, plan->sp, 0, g, s);
      if (e == hipSuccess) e = plan->ks.p_half(vrev, plan->fp, plan->fu, s);            // fp = P_t
      if (e == hipSuccess) e = plan->ks.adj_u_walls(va, gf, u_bar, p_bar, plan->wscr, s);  // Ub -= G^T A^T Pb
    }
    return e == hipSuccess ? HL_OK : hip_fail(e, "hl_adjoint_step: gradient launch");
  }
  if (!grad_kappa) {
    for (int64_t n = 0; n < nsteps; ++n) {
      hipError_t e = plan->ks.adj_p(vb, p_bar, u_bar, s);      // Pb -= B^T Ub
      if (e == hipSuccess) e = plan->ks.adj_u(va, u_bar, p_bar, s);  // Ub -= A^T Pb
      if (e != hipSuccess) return hip_fail(e, "hl_adjoint_step: launch");
    }
    return HL_OK;
  }
  // Gradient: walk the forward state back one step at a time (the step is
  // reversed exactly, in exact arithmetic, by the half-steps with -dt in
  // reverse order) and add each step's contribution
  //   -<Pb' - B^T Ub', A_kappa U_t> - <Ub', B_kappa P'>
  // (the chain rule through P' = P - A U, U' = U - B P').
  if ((st = ensure_gradient(plan)) != HL_OK) return st;
  hl::PlanView vdk = v, vrev = v;
  vdk.tab = plan->tab_dk;
  vrev.tab = plan->tab_rev;
  const size_t pbytes = (size_t)plan->nc * plan->pnodes * state_bytes(plan);
  const size_t ubytes = (size_t)plan->d * plan->nc * plan->unodes * state_bytes(plan);
  double* g = static_cast<double*>(grad_kappa);
  hipError_t e = hipMemcpyAsync(plan->fp, p, pbytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(plan->fu, u, ubytes, hipMemcpyDeviceToDevice, s);
  for (int64_t n = 0; n < nsteps && e == hipSuccess; ++n) {
    // (fp, fu) = (P', U') after the step being undone; (p_bar, u_bar) its adjoint
    e = hipMemsetAsync(plan->su, 0, ubytes, s);
    if (e == hipSuccess) e = plan->ks.u_half(vdk, plan->su, plan->fp, 1.0, s);       // su = -B_kappa P'
    if (e == hipSuccess) e = dot_into(plan, u_bar, plan->su, 1, g, s);
    if (e == hipSuccess) e = plan->ks.u_half(v, plan->fu, plan->fp, -1.0, s);       // fu = U_t
    if (e == hipSuccess) e = plan->ks.adj_p(vb, p_bar, u_bar, s);                    // Pb -= B^T Ub
    if (e == hipSuccess) e = hipMemsetAsync(plan->sp, 0, pbytes, s);
    if (e == hipSuccess) e = plan->ks.p_half(vdk, plan->sp, plan->fu, s);             // sp = -A_kappa U_t
    if (e == hipSuccess) e = dot_into(plan, p_bar, plan->sp, 0, g, s);
    if (e == hipSuccess) e = plan->ks.p_half(vrev, plan->fp, plan->fu, s);            // fp = P_t
    if (e == hipSuccess) e = plan->ks.adj_u(va, u_bar, p_bar, s);                    // Ub -= A^T Pb
  }
  return e == hipSuccess ? HL_OK : hip_fail(e, "hl_adjoint_step: gradient launch");
}

hl_status hl_set_tile(hl_plan_t plan, int32_t tx, int32_t ty, int32_t ygroup) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_set_tile");
  if (st != HL_OK) return st;
  if (tx == 0 && ty == 0) {
    tx = plan->ks.tile[0];
    ty = plan->ks.tile[1];
  }
  if (!valid_tile(plan->d, tx, ty))
    return fail(HL_ERR_ARG, "hl_set_tile: tx a multiple of 32 in [32, 256], ty >= 1 (1 in 1D), 64 <= tx ty <= 256");
  if (ygroup < 0) return fail(HL_ERR_ARG, "hl_set_tile: ygroup must be >= 0");
  hl::Grid gp, gu;
  if (!build_grids(plan, tx, ty, ygroup == 0 ? kYGroup3 : ygroup, &gp, &gu))
    return fail(HL_ERR_UNSUPPORTED, "hl_set_tile: grid too large for the launch");
  hipError_t e = hipDeviceSynchronize();  // launches in flight keep their own grid copies; graphs are rebuilt
  if (e != hipSuccess) return hip_fail(e, "hl_set_tile: pending work failed");
  drop_graph(plan);
  ++plan->gen;
  plan->gp = gp;
  plan->gu = gu;
  plan->ygroup_req = ygroup == 0 ? kYGroup3 : ygroup;
  return HL_OK;
}

hl_status hl_tune(hl_plan_t plan, const void* p, const void* u, int32_t reps, void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_tune");
  if (st != HL_OK) return st;
  if (!p || !u || p == u) return fail(HL_ERR_ARG, "hl_tune: p and u must be distinct non-NULL buffers");
  if (reps < 1) return fail(HL_ERR_ARG, "hl_tune: reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const size_t pbytes = (size_t)plan->nc * plan->pnodes * state_bytes(plan);
  const size_t ubytes = (size_t)plan->d * plan->nc * plan->unodes * state_bytes(plan);
  void *tp = nullptr, *tu = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&tp, pbytes);
  if (e == hipSuccess) e = hipMalloc(&tu, ubytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemcpyAsync(tp, p, pbytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(tu, u, ubytes, hipMemcpyDeviceToDevice, s);
  // candidates: (tx, ty, y-group); the plan's steps run on copies of (p, u)
  std::vector<std::array<int32_t, 3>> cand;
  if (plan->d == 1) {
    for (int32_t tx : {256, 128, 64}) cand.push_back({tx, 1, 1});
  } else {
    const int32_t shapes[][2] = {{64, 4}, {64, 2}, {64, 1}, {128, 2}, {128, 1}, {256, 1}, {32, 8}};
    for (const auto& sh : shapes)
      for (int32_t yg : plan->d == 3 ? std::vector<int32_t>{1, 2, 4} : std::vector<int32_t>{1})
        cand.push_back({sh[0], sh[1], yg});
  }
  float best = -1.0f;
  std::array<int32_t, 3> pick = {plan->ks.tile[0], plan->ks.tile[1], kYGroup3};
  for (size_t c = 0; c < cand.size() && e == hipSuccess; ++c) {
    hl_plan_s trial = *plan;  // grids only; no ownership is taken or released
    if (!build_grids(plan, cand[c][0], cand[c][1], cand[c][2], &trial.gp, &trial.gu)) continue;
    const hl::PlanView v = view(&trial);
    auto one = [&]() -> hipError_t {
      hipError_t le = hipSuccess;
      if (plan->walls) le = plan->ks.ghost(v, tu, s);
      if (le == hipSuccess) le = p_fn(plan)(v, tp, tu, s);
      if (le == hipSuccess) le = u_fn(plan)(v, tu, tp, 1.0, s);
      return le;
    };
    e = one();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = one();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (best < 0.0f || ms < best)) {
      best = ms;
      pick = cand[c];
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (void* q : {tp, tu})
    if (q) (void)hipFree(q);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "hl_tune: trial steps");
  return hl_set_tile(plan, pick[0], pick[1], pick[2]);
}

hl_status hl_adjoint_step_var(hl_plan_t plan, void* p_bar, void* u_bar, const void* p_next, const void* u_prev,
                              void* stream) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_adjoint_step_var");
  if (st != HL_OK) return st;
  if (!plan->var_kappa) return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step_var: the plan has no kappa data (hl_set_kappa)");
  if (!plan->ks.grad_p_var)
    return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step_var: built for d = 1 (all m), d = 2 (m <= 3) and d = 3 "
                                    "(m <= 1)");
  if (!p_bar || !u_bar || !p_next || !u_prev)
    return fail(HL_ERR_ARG, "hl_adjoint_step_var: NULL buffer");
  const void* bufs[4] = {p_bar, u_bar, p_next, u_prev};
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b)
      if (bufs[a] == bufs[b]) return fail(HL_ERR_ARG, "hl_adjoint_step_var: the four buffers must be distinct");
  if ((st = ensure_var_gradient(plan)) != HL_OK) return st;
  hl::PlanView v = view(plan);
  // the gradient kernels run 64 work-items per workgroup (per-lane LDS arrays)
  hl::PlanView v64 = v;
  if (!build_grids(plan, 64, 1, plan->gp.ygroup, &v64.gp, &v64.gu))
    return fail(HL_ERR_ARG, "hl_adjoint_step_var: grid too large");
  hipStream_t s = (hipStream_t)stream;
  if (plan->walls) {
    // The walled step is P' = P - A G U, U' = U - B P' (G the ghost refresh),
    // so: Pb -= B^T Ub from the K dual nodes (dS/dc held on the padded dual
    // array, whose ghost slots stay zero), then Ub -= G^T A^T Pb with A^T on
    // every slot of the padded array and the ghost fold; A_kappa reads G U_t.
    hl::Grid gf;
    const int32_t tile[3] = {plan->gu.tx, plan->gu.ty, 1};
    if (!make_grid(plan, tile, plan->gu.ygroup, plan->uext, plan->uext, 0, plan->pext, -1, plan->unodes,
                   plan->pnodes, &gf))
      return fail(HL_ERR_UNSUPPORTED, "hl_adjoint_step_var: grid too large for the launch");
    const size_t zb = (size_t)kappa_planes(plan) * plan->unodes * plan->tab_bytes;
    const size_t ub = (size_t)plan->d * plan->nc * plan->unodes * state_bytes(plan);
    hipError_t e = hipSuccess;
    for (auto [q, bytes] : {std::pair<void**, size_t>{&plan->vzw, zb}, {&plan->ucw, ub}, {&plan->wscr, ub}}) {
      if (*q) continue;
      e = hipMalloc(q, bytes);
      if (e == hipSuccess) e = hipMemset(*q, 0, bytes);
      if (e != hipSuccess) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
        return fail(HL_ERR_NOMEM, std::string("hl_adjoint_step_var: wall buffers: ") + hipGetErrorString(e));
      }
    }
    e = plan->ks.ghost_zero(v, u_bar, s);
    if (e == hipSuccess) e = plan->ks.grad_u_var(v64, u_bar, p_next, plan->gku, plan->vzw, s);
    if (e == hipSuccess) e = plan->ks.gather_p_var(v, p_bar, plan->vzw, s);               // Pb -= B^T Ub
    if (e == hipSuccess) e = hipMemcpyAsync(plan->ucw, u_prev, ub, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = plan->ks.ghost(v, plan->ucw, s);                             // G U_t
    if (e == hipSuccess) e = plan->ks.grad_p_var(v64, p_bar, plan->ucw, plan->gkp, plan->vscr, s);
    if (e == hipSuccess) e = plan->ks.gather_u_var_walls(v, gf, u_bar, plan->vscr, plan->wscr, s);  // Ub -= G^T A^T Pb
    if (e != hipSuccess) return hip_fail(e, "hl_adjoint_step_var: launch");
    return HL_OK;
  }
  // velocity half-step of the step being undone: gku -= d<Ub, B P'>/dkappa, z = d/dc
  hipError_t e = plan->ks.grad_u_var(v64, u_bar, p_next, plan->gku, plan->vscr, s);
  if (e == hipSuccess) e = plan->ks.gather_p_var(v, p_bar, plan->vscr, s);            // Pb -= B^T Ub
  // pressure half-step: gkp -= d<Pb, A U_t>/dkappa, rho = d/dc
  if (e == hipSuccess) e = plan->ks.grad_p_var(v64, p_bar, u_prev, plan->gkp, plan->vscr, s);
  if (e == hipSuccess) e = plan->ks.gather_u_var(v, u_bar, plan->vscr, s);            // Ub -= A^T Pb
  if (e != hipSuccess) return hip_fail(e, "hl_adjoint_step_var: launch");
  return HL_OK;
}

hl_status hl_kappa_grad(hl_plan_t plan, double* grad_p, double* grad_u, int reset) {
  g_last_error.clear();
  hl_status st = check_plan(plan, "hl_kappa_grad");
  if (st != HL_OK) return st;
  if (!plan->ks.grad_p_var)
    return fail(HL_ERR_UNSUPPORTED, "hl_kappa_grad: built for d = 1 (all m), d = 2 (m <= 3) and d = 3 (m <= 1)");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hl_kappa_grad: pending work failed");
  if ((st = ensure_var_gradient(plan)) != HL_OK) return st;
  const int64_t np = kappa_planes(plan);
  double* dev[2] = {plan->gkp, plan->gku};
  double* host[2] = {grad_p, grad_u};
  const int64_t nodes[2] = {plan->pnodes, plan->unodes};
  for (int f = 0; f < 2; ++f) {
    // hl_set_kappa's layout (with walls: K+1 primal nodes, dual nodes in the padded array)
    const LayoutMap L = hl_host::field_layout(plan->d, 2 * plan->m + 1, plan->K, plan->walls, f);
    if (host[f]) {
      std::vector<double> img((size_t)(np * nodes[f]));
      e = hipMemcpy(img.data(), dev[f], img.size() * sizeof(double), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "hl_kappa_grad: copy to host");
      L.for_each([&](int64_t h, int64_t dv) { host[f][h] = img[(size_t)dv]; });
    }
    if (reset && (e = hipMemset(dev[f], 0, (size_t)(np * nodes[f]) * sizeof(double))) != hipSuccess)
      return hip_fail(e, "hl_kappa_grad: reset");
  }
  return HL_OK;
}

hl_status hl_batch_create(const hl_plan_t* plans, int32_t n, hl_batch_t* out) {
  g_last_error.clear();
  if (!plans || !out || n < 1) return fail(HL_ERR_ARG, "hl_batch_create: need n >= 1 plans and an output handle");
  for (int32_t i = 0; i < n; ++i) {
    hl_status st = check_plan(plans[i], "hl_batch_create");
    if (st != HL_OK) return st;
    const hl_plan_s* p = plans[i];
    if (p->d != plans[0]->d || p->m != plans[0]->m || p->precision != plans[0]->precision)
      return fail(HL_ERR_ARG, "hl_batch_create: every plan must have the same d, m and precision");
  }
  hl_batch_s* b = new (std::nothrow) hl_batch_s();
  if (!b) return fail(HL_ERR_NOMEM, "hl_batch_create: out of host memory");
  b->plans.assign(plans, plans + n);
  for (int32_t i = 0; i < n; ++i) b->walls = b->walls || plans[i]->walls;
  b->ks = plans[0]->ks;
  b->device = plans[0]->device;
  *out = b;
  return HL_OK;
}

hl_status hl_batch_destroy(hl_batch_t batch) {
  g_last_error.clear();
  if (!batch) return HL_OK;
  if (batch->gexec) (void)hipGraphExecDestroy(batch->gexec);
  if (batch->cap_stream) (void)hipStreamDestroy(batch->cap_stream);
  if (batch->dp) (void)hipFree(batch->dp);
  if (batch->du) (void)hipFree(batch->du);
  drop_sources(batch);
  delete batch;
  return HL_OK;
}

hl_status hl_batch_set_sources(hl_batch_t batch, const int64_t* counts, const int64_t* const* nodes,
                               const double* const* values, const double* const* amps, int64_t namps) {
  g_last_error.clear();
  if (!batch) return fail(HL_ERR_ARG, "hl_batch_set_sources: batch is NULL");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hl_batch_set_sources: pending work failed");
  if (batch->gexec) (void)hipGraphExecDestroy(batch->gexec);
  batch->gexec = nullptr;
  batch->bp.clear();  // the next hl_batch_step rebuilds its tables
  drop_sources(batch);
  if (!counts) return HL_OK;
  if (!batch->ks.batch_src) return fail(HL_ERR_UNSUPPORTED, "hl_batch_set_sources: not built for this batch");
  if (namps < 0 || !nodes || !values || !amps) return fail(HL_ERR_ARG, "hl_batch_set_sources: bad arguments");
  const int n = (int)batch->plans.size();
  const hl_plan_s* p0 = batch->plans[0];
  const int d = p0->d, mp = p0->m + 1, nc = p0->nc;
  // values and amplitudes in the storage's arithmetic type: FP64 words for
  // FP64 and FP32_COMP (whose values are first rounded to hi + lo, as the
  // split storage would hold g), FP32 words for FP32
  const bool f64 = p0->precision != HL_FP32, split = p0->precision == HL_FP32_COMP;
  std::vector<hl::BatchSource> ent;
  std::vector<double> val, amp((size_t)n * (size_t)namps, 0.0);
  for (int i = 0; i < n; ++i) {
    if (counts[i] < 0) return fail(HL_ERR_ARG, "hl_batch_set_sources: negative count");
    if (counts[i] == 0) continue;
    if (!nodes[i] || !values[i]) return fail(HL_ERR_ARG, "hl_batch_set_sources: NULL node or value array");
    const hl_plan_s* pl = batch->plans[i];
    if ((int64_t)nc * pl->pnodes > (int64_t)UINT32_MAX)
      return fail(HL_ERR_UNSUPPORTED, "hl_batch_set_sources: pressure array too large for 32-bit word offsets");
    int64_t hn = 1;  // primal nodes (K + 1 per dimension with walls)
    for (int k = 0; k < d; ++k) hn *= pl->pext[k];
    // distinct nodes: each entry's update is a plain read-modify-write
    std::vector<int64_t> sorted(nodes[i], nodes[i] + counts[i]);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(HL_ERR_ARG, "hl_batch_set_sources: a shot's source nodes must be distinct");
    for (int64_t q = 0; q < counts[i]; ++q) {
      int64_t flat = nodes[i][q];
      if (flat < 0 || flat >= hn) return fail(HL_ERR_ARG, "hl_batch_set_sources: node index out of range");
      int64_t j[3] = {0, 0, 0};
      for (int k = d - 1; k >= 0; --k) {  // host order: j_1 slowest
        j[k] = flat % pl->pext[k];
        flat /= pl->pext[k];
      }
      const int64_t dn = j[0] + (int64_t)pl->pext[0] * (j[1] + (int64_t)pl->pext[1] * j[2]);
      for (int c = 0; c < nc; ++c) {
        int a[3] = {0, 0, 0}, r = c;
        for (int k = d - 1; k >= 0; --k) {  // host coefficient order: a_1 slowest
          a[k] = r % mp;
          r /= mp;
        }
        const int plane = a[0] + mp * (a[1] + mp * a[2]);
        const double v = values[i][q * nc + c];
        if (!std::isfinite(v)) return fail(HL_ERR_ARG, "hl_batch_set_sources: values must be finite");
        ent.push_back(hl::BatchSource{(int32_t)i, (uint32_t)(plane * pl->pnodes + dn)});
        if (split) {
          hl_host::FieldImage one{HL_FP32_COMP, 1, {}, {}};
          if (!one.alloc()) return fail(HL_ERR_NOMEM, "hl_batch_set_sources: out of host memory");
          one.put(0, v);
          val.push_back(one.get(0));
        } else {
          val.push_back(v);
        }
      }
    }
    if (amps[i])
      for (int64_t t = 0; t < namps; ++t) {
        if (!std::isfinite(amps[i][t])) return fail(HL_ERR_ARG, "hl_batch_set_sources: amplitudes must be finite");
        amp[(size_t)i * namps + t] = amps[i][t];
      }
  }
  const size_t wb = f64 ? 8 : 4;
  auto words = [&](const std::vector<double>& v) {
    std::vector<unsigned char> out(std::max<size_t>(v.size(), 1) * wb, 0);
    for (size_t k = 0; k < v.size(); ++k) {
      if (f64) {
        std::memcpy(out.data() + 8 * k, &v[k], 8);
      } else {
        const float x = (float)v[k];
        std::memcpy(out.data() + 4 * k, &x, 4);
      }
    }
    return out;
  };
  const std::vector<unsigned char> vw = words(val), aw = words(amp);
  const int64_t zero = 0;
  e = hipMalloc(&batch->d_pbase, (size_t)(split ? 2 : 1) * n * sizeof(void*));
  if (e == hipSuccess) e = hipMalloc(&batch->d_ent, std::max<size_t>(ent.size(), 1) * sizeof(hl::BatchSource));
  if (e == hipSuccess) e = hipMalloc(&batch->d_val, vw.size());
  if (e == hipSuccess) e = hipMalloc(&batch->d_amps, aw.size());
  if (e == hipSuccess) e = hipMalloc((void**)&batch->d_counter, sizeof(int64_t));
  if (e != hipSuccess) {
    drop_sources(batch);
    return fail(HL_ERR_NOMEM, "hl_batch_set_sources: device allocation failed");
  }
  if (!ent.empty()) e = hipMemcpy(batch->d_ent, ent.data(), ent.size() * sizeof(hl::BatchSource), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(batch->d_val, vw.data(), vw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(batch->d_amps, aw.data(), aw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(batch->d_counter, &zero, sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    drop_sources(batch);
    return hip_fail(e, "hl_batch_set_sources: upload");
  }
  batch->nent = (int64_t)ent.size();
  batch->namps = namps;
  batch->src = true;
  return HL_OK;
}

hl_status hl_batch_step(hl_batch_t batch, void* const* p, void* const* u, int64_t nsteps, void* stream) {
  g_last_error.clear();
  if (!batch) return fail(HL_ERR_ARG, "hl_batch_step: batch is NULL");
  if (!p || !u) return fail(HL_ERR_ARG, "hl_batch_step: NULL buffer arrays");
  if (nsteps < 0) return fail(HL_ERR_ARG, "hl_batch_step: nsteps must be >= 0");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != batch->device)
    return fail(HL_ERR_DEVICE, "hl_batch_step: current HIP device differs from the batch's device");
  const int n = (int)batch->plans.size();
  const bool var = batch->plans[0]->var_kappa;
  for (int i = 0; i < n; ++i) {
    if (!p[i] || !u[i] || p[i] == u[i]) return fail(HL_ERR_ARG, "hl_batch_step: p[i] and u[i] must be distinct non-NULL");
    if (batch->plans[i]->var_kappa != var)
      return fail(HL_ERR_ARG, "hl_batch_step: variable kappa must be set on every plan of the batch or on none");
  }
  if (var && !batch->ks.batch_var)
    return fail(HL_ERR_UNSUPPORTED, "hl_batch_step: batched variable kappa is not built for this (d, m)");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  bool same = var == batch->var && batch->bp.size() == (size_t)n && batch->gens.size() == (size_t)n &&
              std::equal(batch->bp.begin(), batch->bp.end(), p) && std::equal(batch->bu.begin(), batch->bu.end(), u);
  for (int i = 0; i < n && same; ++i) same = batch->gens[i] == batch->plans[i]->gen;
  if (!same) {
    // descriptors for these buffers; wait for work that may still read the old ones
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hl_batch_step: pending work failed");
    if (batch->gexec) (void)hipGraphExecDestroy(batch->gexec);
    batch->gexec = nullptr;
    std::vector<hl::PlanView> views((size_t)n);
    std::vector<hl::BatchShot> shots((size_t)n);
    // the batched launch has one workgroup shape: the shots' own tile when
    // they all share one (hl_set_tile / hl_tune), else the default
    bool common = true;
    const hl_plan_s* p0 = batch->plans[0];
    for (int i = 1; i < n; ++i) {
      const hl_plan_s* pi = batch->plans[i];
      common = common && pi->gp.tx == p0->gp.tx && pi->gp.ty == p0->gp.ty && pi->ygroup_req == p0->ygroup_req;
    }
    batch->tile[0] = common ? p0->gp.tx : batch->ks.tile[0];
    batch->tile[1] = common ? p0->gp.ty : batch->ks.tile[1];
    batch->tile[2] = common ? p0->ygroup_req : kYGroup3;
    for (int i = 0; i < n; ++i) {
      const hl_plan_s* pl = batch->plans[i];
      views[i] = view(pl);
      if (!build_grids(pl, batch->tile[0], batch->tile[1], batch->tile[2], &views[i].gp, &views[i].gu))
        return fail(HL_ERR_UNSUPPORTED, "hl_batch_step: grid too large for the launch");
      shots[i] = hl::BatchShot{&views[i], p[i], u[i]};
    }
    std::vector<unsigned char> pd, ud;
    batch->ks.batch_desc(shots.data(), n, var, &pd, &ud, &batch->pblocks, &batch->ublocks);
    if (pd.size() > batch->cap) {
      if (batch->dp) (void)hipFree(batch->dp);
      if (batch->du) (void)hipFree(batch->du);
      batch->dp = batch->du = nullptr;
      batch->cap = 0;
      e = hipMalloc(&batch->dp, pd.size());
      if (e == hipSuccess) e = hipMalloc(&batch->du, ud.size());
      if (e != hipSuccess) return fail(HL_ERR_NOMEM, "hl_batch_step: descriptor allocation failed");
      batch->cap = pd.size();
    }
    e = hipMemcpy(batch->dp, pd.data(), pd.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(batch->du, ud.data(), ud.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hl_batch_step: descriptor upload");
    if (batch->src) {
      if (batch->plans[0]->precision == HL_FP32_COMP) {  // hi and lo bases per shot
        std::vector<void*> hl2((size_t)2 * n);
        for (int i = 0; i < n; ++i) {
          hl2[2 * i] = p[i];
          hl2[2 * i + 1] = static_cast<char*>(p[i]) + (size_t)4 * batch->plans[i]->nc * batch->plans[i]->pnodes;
        }
        e = hipMemcpy(batch->d_pbase, hl2.data(), hl2.size() * sizeof(void*), hipMemcpyHostToDevice);
      } else {
        e = hipMemcpy(batch->d_pbase, p, (size_t)n * sizeof(void*), hipMemcpyHostToDevice);
      }
      if (e != hipSuccess) return hip_fail(e, "hl_batch_step: source buffer table upload");
    }
    batch->bp.assign(p, p + n);
    batch->bu.assign(u, u + n);
    batch->gens.resize((size_t)n);
    for (int i = 0; i < n; ++i) batch->gens[i] = batch->plans[i]->gen;
    batch->views = views;
    batch->var = var;
  }
  auto one_step = [&](hipStream_t st) -> hipError_t {
    hipError_t le = hipSuccess;
    // walled shots: refresh their ghost velocity before the pressure half-step
    for (int i = 0; i < n && le == hipSuccess && batch->walls; ++i)
      if (batch->plans[i]->walls) le = batch->ks.ghost(batch->views[i], u[i], st);
    const dim3 block((unsigned)batch->tile[0], (unsigned)batch->tile[1], 1);
    if (le == hipSuccess) le = batch->ks.p_batch(batch->dp, n, batch->pblocks, var, block, st);
    if (le == hipSuccess && batch->src) {
      le = batch->ks.batch_src(batch->d_pbase, batch->d_ent, batch->d_val, batch->d_amps, batch->namps,
                               batch->d_counter, batch->nent, st);
      if (le == hipSuccess) {
        hipLaunchKernelGGL(batch_tick, dim3(1), dim3(64), 0, st, batch->d_counter);
        le = hipGetLastError();
      }
    }
    if (le == hipSuccess) le = batch->ks.u_batch(batch->du, n, batch->ublocks, var, block, st);
    return le;
  };
  int64_t k = 0;
  if (nsteps >= kGraphChunk) {
    if (!batch->gexec) {
      if (!batch->cap_stream && (e = hipStreamCreateWithFlags(&batch->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hl_batch_step: stream");
      if ((e = hipStreamBeginCapture(batch->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hl_batch_step: capture");
      hipError_t le = hipSuccess;
      for (int64_t i = 0; i < kGraphChunk && le == hipSuccess; ++i) le = one_step(batch->cap_stream);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(batch->cap_stream, &graph);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&batch->gexec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        batch->gexec = nullptr;
        return hip_fail(e, "hl_batch_step: graph capture");
      }
    }
    for (; k + kGraphChunk <= nsteps; k += kGraphChunk)
      if ((e = hipGraphLaunch(batch->gexec, s)) != hipSuccess) return hip_fail(e, "hl_batch_step: graph launch");
  }
  for (; k < nsteps; ++k)
    if ((e = one_step(s)) != hipSuccess) return hip_fail(e, "hl_batch_step: launch");
  return HL_OK;
}

}  // extern "C"
