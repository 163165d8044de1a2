// Oracle: a plain, slow, arbitrary-precision CPU simulator of the time-dependent
// matrix-product-state method of SaiToh's ZKCM_QC report (arXiv:1111.3124).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code, header,
// table or helper with the device library; the two meet only in the seeded
// inputs drawn by paper_1111_3124_amd/workloads.py.
//
// What it follows:
//  * The state |Psi> = sum c_{i0..i(n-1)} |i0..i(n-1)>, normalised (Section 3.1).
//  * Eq. (1): the MPS form Q_0 V_0 Q_1 V_1 ... V_{n-2} Q_{n-1}, kept literally as
//    Vidal's Gamma-lambda form (Gamma_s == Q_s, lambda_s == V_s), with Q_s holding
//    2 x m_{s-1} x m_s entries.
//  * Eq. (2): V_s are the Schmidt coefficients across the cut s | s+1, stored
//    sorted, with sum V_s^2 = 1.
//  * Section 3.1: a U(4) gate on qubits s, s+1 updates Q_s, V_s, Q_{s+1} only;
//    small Schmidt coefficients are truncated; U(2) and U(8) gates are elementary.
//    The update itself is Vidal's (the reference the paper defers to):
//      theta = lambda_{s-1} Gamma_s lambda_s Gamma_{s+1} lambda_{s+1} mixed by U,
//      theta = X Sigma Z^H,  lambda_s' = sigma / nu,
//      Gamma_s' = lambda_{s-1}^{-1} X,  Gamma_{s+1}' = Z^H lambda_{s+1}^{-1}.
//    A U(8) gate splits left first (s | s+1 s+2), then (s+1 | s+2).
//  * The SVD is a one-sided (Hestenes) Jacobi iteration on the columns of theta,
//    each rotation the complex form of the symmetric 2x2 Schur decomposition
//    (Golub and Van Loan, Matrix Computations, sections 8.5 and 8.6), pairs visited
//    in round-robin order so that the pairs of one round are disjoint.
//  * Truncation (the paper gives no threshold): with sigma sorted descending and
//    W = sum sigma_j^2, k_eps is the smallest k >= 1 whose discarded weight
//    sum_{j>=k} sigma_j^2 is <= eps * W; k = min(chi_max, k_eps, rank), where rank
//    counts sigma_j > 2^{-(prec-36)} sigma_1.  Kept values are renormalised.
//
// All arithmetic is MPFR at `prec` bits (256 by default: the precision of the
// paper's own MPS example), round-to-nearest.  Inputs arrive as binary64 or as
// exact double-double pairs; outputs leave as (hi, lo) pairs.
//
//  * Reduced density operators (Section 3.2's RDO_block / RDO(list)): the partial
//    trace of |Psi><Psi| over the unlisted qubits, contracted site by site.
//
// Parity pins (the tests in tests/test_oracle_*.py): the paper's 3-qubit example
// (amplitudes and its printed RDOs), GHZ and QFT closed forms, a dense state vector
// for <= 12 qubits, SVD identities checked outside this file, Eckart-Young, the
// invariants sum lambda^2 = 1, and RDOs against a textbook partial trace, product
// and GHZ closed forms and Tr rho = 1.

#include <mpfr.h>
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

namespace {

const mpfr_rnd_t RN = MPFR_RNDN;
int g_prec = 256;  // precision of every temporary created by the current call

struct Re {
  mpfr_t v;
  Re() { mpfr_init2(v, g_prec); mpfr_set_ui(v, 0, RN); }
  Re(const Re& o) { mpfr_init2(v, mpfr_get_prec(o.v)); mpfr_set(v, o.v, RN); }
  Re(Re&& o) noexcept { mpfr_init2(v, mpfr_get_prec(o.v)); mpfr_swap(v, o.v); }
  Re& operator=(const Re& o) {
    if (this != &o) { mpfr_set_prec(v, mpfr_get_prec(o.v)); mpfr_set(v, o.v, RN); }
    return *this;
  }
  Re& operator=(Re&& o) noexcept { mpfr_swap(v, o.v); return *this; }
  ~Re() { mpfr_clear(v); }
};

struct Cx { Re re, im; };

using CVec = std::vector<Cx>;

// dense complex matrix, column-major
struct CMat {
  int rows = 0, cols = 0;
  CVec a;
  CMat() {}
  CMat(int r, int c) : rows(r), cols(c), a((size_t)r * c) {}
  Cx& at(int r, int c) { return a[(size_t)c * rows + r]; }
  const Cx& at(int r, int c) const { return a[(size_t)c * rows + r]; }
  Cx* col(int c) { return &a[(size_t)c * rows]; }
};

// per-thread scratch for the inner loops (MPFR temporaries are costly to create)
struct Scratch {
  Re t[8];
  Re al, be, gabs, zeta, tt, c, sn, tmp;
  Cx g, e;
};

void set_d2(mpfr_t x, double hi, double lo) {
  mpfr_set_d(x, hi, RN);
  if (lo != 0.0) {
    mpfr_t t; mpfr_init2(t, 64); mpfr_set_d(t, lo, RN);
    mpfr_add(x, x, t, RN);  // exact at >= 2*53+... bits for a valid dd pair
    mpfr_clear(t);
  }
}

void get_d2(const mpfr_t x, double* hi, double* lo) {
  double h = mpfr_get_d(x, RN);
  mpfr_t t; mpfr_init2(t, mpfr_get_prec(x));
  mpfr_sub_d(t, x, h, RN);
  *hi = h;
  *lo = mpfr_get_d(t, RN);
  mpfr_clear(t);
}

// z += x * y  (complex)
void cfma(Cx& z, const Cx& x, const Cx& y, Scratch& s) {
  mpfr_fma(z.re.v, x.re.v, y.re.v, z.re.v, RN);
  mpfr_mul(s.t[0].v, x.im.v, y.im.v, RN);
  mpfr_sub(z.re.v, z.re.v, s.t[0].v, RN);
  mpfr_fma(z.im.v, x.re.v, y.im.v, z.im.v, RN);
  mpfr_fma(z.im.v, x.im.v, y.re.v, z.im.v, RN);
}

// z += x * conj(y)  (complex)
void cfma_cj(Cx& z, const Cx& x, const Cx& y, Scratch& s) {
  mpfr_fma(z.re.v, x.re.v, y.re.v, z.re.v, RN);
  mpfr_fma(z.re.v, x.im.v, y.im.v, z.re.v, RN);
  mpfr_fma(z.im.v, x.im.v, y.re.v, z.im.v, RN);
  mpfr_mul(s.t[0].v, x.re.v, y.im.v, RN);
  mpfr_sub(z.im.v, z.im.v, s.t[0].v, RN);
}

// z = x * y (complex), z distinct from x and y
void cmul(Cx& z, const Cx& x, const Cx& y, Scratch& s) {
  mpfr_mul(z.re.v, x.re.v, y.re.v, RN);
  mpfr_mul(s.t[0].v, x.im.v, y.im.v, RN);
  mpfr_sub(z.re.v, z.re.v, s.t[0].v, RN);
  mpfr_mul(z.im.v, x.re.v, y.im.v, RN);
  mpfr_fma(z.im.v, x.im.v, y.re.v, z.im.v, RN);
}

// ---------------------------------------------------------------- Jacobi SVD
//
// One-sided Jacobi on the columns of A (M x N): A <- A V with V unitary, until
// every pair of columns is orthogonal to working precision.  On return the
// columns of A are W = A_in V, sigma_j = ||W_j||.
struct SvdResult {
  int sweeps = 0;
  bool converged = false;
};

// Gram entries of columns x, y:  al = ||x||^2, be = ||y||^2, g = x^H y
void gram2(const Cx* x, const Cx* y, int m, Re& al, Re& be, Cx& g, Scratch& s) {
  mpfr_set_ui(al.v, 0, RN); mpfr_set_ui(be.v, 0, RN);
  mpfr_set_ui(g.re.v, 0, RN); mpfr_set_ui(g.im.v, 0, RN);
  mpfr_set_ui(s.t[1].v, 0, RN);
  for (int i = 0; i < m; ++i) {
    mpfr_fma(al.v, x[i].re.v, x[i].re.v, al.v, RN);
    mpfr_fma(al.v, x[i].im.v, x[i].im.v, al.v, RN);
    mpfr_fma(be.v, y[i].re.v, y[i].re.v, be.v, RN);
    mpfr_fma(be.v, y[i].im.v, y[i].im.v, be.v, RN);
    // conj(x) * y = (xr yr + xi yi) + i (xr yi - xi yr)
    mpfr_fma(g.re.v, x[i].re.v, y[i].re.v, g.re.v, RN);
    mpfr_fma(g.re.v, x[i].im.v, y[i].im.v, g.re.v, RN);
    mpfr_fma(g.im.v, x[i].re.v, y[i].im.v, g.im.v, RN);
    mpfr_fma(s.t[1].v, x[i].im.v, y[i].re.v, s.t[1].v, RN);
  }
  mpfr_sub(g.im.v, g.im.v, s.t[1].v, RN);
}

// [x, y] <- [x, y] [[c, s], [-s e, c e]] with e = e^{-i phi}:
//   x' = c x - s e y,  y' = s x + c e y
void rot2(Cx* x, Cx* y, int m, const Re& c, const Re& sn, const Cx& e, Scratch& s) {
  Re& eyr = s.t[2]; Re& eyi = s.t[3]; Re& u = s.t[4]; Re& w = s.t[5];
  for (int i = 0; i < m; ++i) {
    // ey = e * y
    mpfr_mul(eyr.v, e.re.v, y[i].re.v, RN);
    mpfr_mul(u.v, e.im.v, y[i].im.v, RN);
    mpfr_sub(eyr.v, eyr.v, u.v, RN);
    mpfr_mul(eyi.v, e.re.v, y[i].im.v, RN);
    mpfr_fma(eyi.v, e.im.v, y[i].re.v, eyi.v, RN);
    // y' = s x + c ey ; x' = c x - s ey
    mpfr_mul(u.v, sn.v, x[i].re.v, RN);
    mpfr_fma(u.v, c.v, eyr.v, u.v, RN);
    mpfr_mul(w.v, sn.v, x[i].im.v, RN);
    mpfr_fma(w.v, c.v, eyi.v, w.v, RN);
    mpfr_mul(x[i].re.v, c.v, x[i].re.v, RN);
    mpfr_mul(eyr.v, sn.v, eyr.v, RN);
    mpfr_sub(x[i].re.v, x[i].re.v, eyr.v, RN);
    mpfr_mul(x[i].im.v, c.v, x[i].im.v, RN);
    mpfr_mul(eyi.v, sn.v, eyi.v, RN);
    mpfr_sub(x[i].im.v, x[i].im.v, eyi.v, RN);
    mpfr_set(y[i].re.v, u.v, RN);
    mpfr_set(y[i].im.v, w.v, RN);
  }
}

// One Jacobi rotation on columns p, q of A (and of V).  Returns true if rotated.
// Columns whose squared norm is <= ztol (rounding level of the whole matrix) are
// numerically zero: they are left alone, since no rotation can make noise
// orthogonal to itself in relative terms.
bool jacobi_pair(CMat& A, CMat& V, int p, int q, const Re& tol, const Re& ztol, Scratch& s) {
  Re& al = s.al; Re& be = s.be; Re& gabs = s.gabs; Re& zeta = s.zeta; Re& t = s.tt;
  Re& c = s.c; Re& sn = s.sn; Re& tmp = s.tmp;
  Cx& g = s.g; Cx& e = s.e;
  gram2(A.col(p), A.col(q), A.rows, al, be, g, s);
  if (mpfr_cmp(al.v, ztol.v) <= 0 || mpfr_cmp(be.v, ztol.v) <= 0) return false;
  mpfr_hypot(gabs.v, g.re.v, g.im.v, RN);
  // rotate only if |g| > tol * sqrt(al * be)
  mpfr_mul(tmp.v, al.v, be.v, RN);
  mpfr_sqrt(tmp.v, tmp.v, RN);
  mpfr_mul(tmp.v, tmp.v, tol.v, RN);
  if (mpfr_cmp(gabs.v, tmp.v) <= 0) return false;
  // zeta = (be - al) / (2|g|);  t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2))
  mpfr_sub(zeta.v, be.v, al.v, RN);
  mpfr_div(zeta.v, zeta.v, gabs.v, RN);
  mpfr_div_ui(zeta.v, zeta.v, 2, RN);
  mpfr_sqr(tmp.v, zeta.v, RN);
  mpfr_add_ui(tmp.v, tmp.v, 1, RN);
  mpfr_sqrt(tmp.v, tmp.v, RN);
  mpfr_abs(t.v, zeta.v, RN);
  mpfr_add(t.v, t.v, tmp.v, RN);
  mpfr_ui_div(t.v, 1, t.v, RN);
  if (mpfr_sgn(zeta.v) < 0) mpfr_neg(t.v, t.v, RN);
  // c = 1/sqrt(1+t^2), s = t c
  mpfr_sqr(tmp.v, t.v, RN);
  mpfr_add_ui(tmp.v, tmp.v, 1, RN);
  mpfr_rec_sqrt(c.v, tmp.v, RN);
  mpfr_mul(sn.v, t.v, c.v, RN);
  // e = e^{-i phi} = conj(g) / |g|
  mpfr_div(e.re.v, g.re.v, gabs.v, RN);
  mpfr_div(e.im.v, g.im.v, gabs.v, RN);
  mpfr_neg(e.im.v, e.im.v, RN);
  rot2(A.col(p), A.col(q), A.rows, c, sn, e, s);
  rot2(V.col(p), V.col(q), V.rows, c, sn, e, s);
  return true;
}

// round-robin ("circle") schedule: rounds of disjoint pairs covering all pairs once
std::vector<std::vector<std::pair<int, int>>> round_robin(int n) {
  int np = n + (n & 1);
  std::vector<int> pos(np);
  for (int i = 0; i < np; ++i) pos[i] = i;
  std::vector<std::vector<std::pair<int, int>>> rounds;
  for (int r = 0; r < np - 1; ++r) {
    std::vector<std::pair<int, int>> pr;
    for (int i = 0; i < np / 2; ++i) {
      int a = pos[i], b = pos[np - 1 - i];
      if (a < n && b < n) pr.emplace_back(std::min(a, b), std::max(a, b));
    }
    rounds.push_back(pr);
    // keep pos[0], rotate the rest by one
    int last = pos[np - 1];
    for (int i = np - 1; i > 1; --i) pos[i] = pos[i - 1];
    pos[1] = last;
  }
  return rounds;
}

int g_max_sweeps = 80;

SvdResult jacobi_svd(CMat& A, CMat& V) {
  const int N = A.cols;
  V = CMat(N, N);
  for (int j = 0; j < N; ++j) mpfr_set_ui(V.at(j, j).re.v, 1, RN);
  SvdResult res;
  if (N < 2) { res.converged = true; return res; }
  Re tol;
  mpfr_set_ui(tol.v, 1, RN);
  mpfr_div_2si(tol.v, tol.v, g_prec - 16, RN);
  // ztol = (2^{-(prec-8)} ||A||_F)^2
  Re ztol;
  for (auto& x : A.a) {
    mpfr_fma(ztol.v, x.re.v, x.re.v, ztol.v, RN);
    mpfr_fma(ztol.v, x.im.v, x.im.v, ztol.v, RN);
  }
  mpfr_div_2si(ztol.v, ztol.v, 2 * (g_prec - 8), RN);
  auto rounds = round_robin(N);
  const bool par = (size_t)A.rows * N >= 4096;
  int nth = par ? omp_get_max_threads() : 1;
  std::vector<Scratch> scr(nth);
  for (int sw = 0; sw < g_max_sweeps; ++sw) {
    int rotated = 0;
    for (auto& pr : rounds) {
      const int np = (int)pr.size();
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rotated) if (par)
      for (int i = 0; i < np; ++i) {
        int th = par ? omp_get_thread_num() : 0;
        if (jacobi_pair(A, V, pr[i].first, pr[i].second, tol, ztol, scr[th])) rotated |= 1;
      }
    }
    res.sweeps = sw + 1;
    if (!rotated) { res.converged = true; break; }
  }
  return res;
}

// ---------------------------------------------------------------- truncation
struct SplitStats {
  double W_hi = 0, W_lo = 0;    // total weight sum sigma^2 before truncation
  double w_hi = 0, w_lo = 0;    // relative discarded weight
  int k = 0, sweeps = 0, rank = 0;
  double gap = INFINITY;        // (sigma_{k-1} - sigma_k) / sigma_0 when a non-zero value is cut
  double epsdist = INFINITY;    // relative distance of the eps decision to its boundary
  int converged = 1;
};

struct Decomp {
  // theta = X diag(sigma) Z^H with sigma sorted descending; r = min(M, N) triplets
  CMat X, Z;               // M x r, N x r
  std::vector<Re> sigma;   // r
  int k = 0;
  Re nu;                   // sqrt(sum_{j<k} sigma_j^2)
  SplitStats st;
};

void column_norms(CMat& A, std::vector<Re>& sig) {
  sig.assign(A.cols, Re());
  for (int j = 0; j < A.cols; ++j) {
    Cx* x = A.col(j);
    for (int i = 0; i < A.rows; ++i) {
      mpfr_fma(sig[j].v, x[i].re.v, x[i].re.v, sig[j].v, RN);
      mpfr_fma(sig[j].v, x[i].im.v, x[i].im.v, sig[j].v, RN);
    }
    mpfr_sqrt(sig[j].v, sig[j].v, RN);
  }
}

// SVD by one-sided Jacobi along the shorter dimension:
//  * M >= N: Jacobi on the columns of A:  A V = W,  X = W / sigma, Z = V;
//  * M <  N: Jacobi on the columns of A^H: A^H V' = W', so A = V' Sigma (W'/sigma)^H:
//            X = V', Z = W' / sigma.
// X or Z columns belonging to sigma = 0 are left zero (never kept by the rank rule).
void svd_xz(const CMat& A, Decomp& d) {
  const int M = A.rows, N = A.cols;
  const bool wide = M < N;
  CMat B, V;
  if (!wide) {
    B = A;
  } else {
    B = CMat(N, M);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < N; ++j) {
        B.at(j, i).re = A.at(i, j).re;
        B.at(j, i).im = A.at(i, j).im;
        mpfr_neg(B.at(j, i).im.v, B.at(j, i).im.v, RN);
      }
  }
  SvdResult r = jacobi_svd(B, V);
  d.st.sweeps = r.sweeps;
  d.st.converged = r.converged;
  std::vector<Re> sig;
  column_norms(B, sig);
  const int R = B.cols;  // == min(M, N)
  std::vector<int> order(R);
  for (int j = 0; j < R; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return mpfr_cmp(sig[x].v, sig[y].v) > 0; });
  d.sigma.assign(R, Re());
  for (int j = 0; j < R; ++j) d.sigma[j] = sig[order[j]];
  CMat& Wc = wide ? d.Z : d.X;   // the side obtained as W / sigma
  CMat& Vc = wide ? d.X : d.Z;   // the side obtained as the accumulated rotations
  Wc = CMat(B.rows, R);
  Vc = CMat(V.rows, R);
  for (int j = 0; j < R; ++j) {
    const int c = order[j];
    const bool nz = !mpfr_zero_p(d.sigma[j].v);
    for (int i = 0; i < B.rows; ++i) {
      if (nz) {
        mpfr_div(Wc.at(i, j).re.v, B.at(i, c).re.v, d.sigma[j].v, RN);
        mpfr_div(Wc.at(i, j).im.v, B.at(i, c).im.v, d.sigma[j].v, RN);
      }
    }
    for (int i = 0; i < V.rows; ++i) Vc.at(i, j) = V.at(i, c);
  }
}

// SVD + rank guard + truncation rule.
Decomp decompose(const CMat& A, int chi_max, double eps) {
  Decomp d;
  svd_xz(A, d);
  const int R = (int)d.sigma.size();
  // tail[k] = sum_{j>=k} sigma_j^2
  std::vector<Re> tail(R + 1);
  for (int j = R - 1; j >= 0; --j) {
    mpfr_sqr(tail[j].v, d.sigma[j].v, RN);
    mpfr_add(tail[j].v, tail[j].v, tail[j + 1].v, RN);
  }
  Re Wt = tail[0];
  get_d2(Wt.v, &d.st.W_hi, &d.st.W_lo);
  // rank guard
  Re guard;
  mpfr_set_ui(guard.v, 1, RN);
  mpfr_div_2si(guard.v, guard.v, g_prec - 36, RN);
  mpfr_mul(guard.v, guard.v, d.sigma[0].v, RN);
  int rank = 0;
  for (int j = 0; j < R; ++j)
    if (mpfr_cmp(d.sigma[j].v, guard.v) > 0) ++rank;
  d.st.rank = rank;
  // eps rule
  Re epsW;
  mpfr_set_d(epsW.v, eps, RN);
  mpfr_mul(epsW.v, epsW.v, Wt.v, RN);
  int keps = R;
  for (int k = 1; k <= R; ++k)
    if (mpfr_cmp(tail[k].v, epsW.v) <= 0) { keps = k; break; }
  int k = std::min(std::min(chi_max, keps), rank);
  if (k < 1) k = 1;
  d.k = k;
  d.st.k = k;
  // nu = sqrt of the kept weight, summed directly (not W - tail, which cancels)
  {
    Re s2, q;
    for (int j = 0; j < k; ++j) { mpfr_sqr(q.v, d.sigma[j].v, RN); mpfr_add(s2.v, s2.v, q.v, RN); }
    mpfr_sqrt(d.nu.v, s2.v, RN);
  }
  {
    Re w; mpfr_div(w.v, tail[k].v, Wt.v, RN);
    get_d2(w.v, &d.st.w_hi, &d.st.w_lo);
  }
  // ambiguity diagnostics
  if (k < rank) {
    Re g; mpfr_sub(g.v, d.sigma[k - 1].v, d.sigma[k].v, RN);
    mpfr_div(g.v, g.v, d.sigma[0].v, RN);
    d.st.gap = mpfr_get_d(g.v, RN);
  }
  if (eps > 0) {
    double best = INFINITY;
    for (int kk : {keps - 1, keps}) {
      if (kk < 1 || kk > R) continue;
      Re dd; mpfr_sub(dd.v, tail[kk].v, epsW.v, RN); mpfr_abs(dd.v, dd.v, RN);
      mpfr_div(dd.v, dd.v, epsW.v, RN);
      best = std::min(best, mpfr_get_d(dd.v, RN));
    }
    d.st.epsdist = best;
  }
  return d;
}

// ---------------------------------------------------------------- MPS (Gamma-lambda)
struct Site {
  int ml = 1, mr = 1;
  CVec g;  // Gamma[(alpha*2 + i)*mr + beta]
  Cx& at(int al, int i, int be) { return g[((size_t)al * 2 + i) * mr + be]; }
};

struct Mps {
  int n, chi_max, prec;
  double eps;
  std::vector<Site> site;
  std::vector<std::vector<Re>> lam;  // lam[s], s = 0..n-2
  SplitStats last[2];
  int nsplits = 0;
  std::string err;
};

// lambda_{s} with the boundary convention lambda_{-1} = lambda_{n-1} = [1]
const Re& lam_at(Mps& m, int s, int idx, const Re& one) {
  if (s < 0 || s >= m.n - 1) return one;
  return m.lam[s][idx];
}

void gate_mix(const std::vector<Cx>& U, int dim, std::vector<Cx>& in, std::vector<Cx>& out,
              Scratch& s) {
  for (int r = 0; r < dim; ++r) {
    mpfr_set_ui(out[r].re.v, 0, RN); mpfr_set_ui(out[r].im.v, 0, RN);
    for (int c = 0; c < dim; ++c) cfma(out[r], U[(size_t)r * dim + c], in[c], s);
  }
}

std::vector<Cx> load_gate(int k, const double* hi, const double* lo) {
  int d = 1 << k;
  std::vector<Cx> U((size_t)d * d);
  for (int i = 0; i < d * d; ++i) {
    set_d2(U[i].re.v, hi[2 * i], lo ? lo[2 * i] : 0.0);
    set_d2(U[i].im.v, hi[2 * i + 1], lo ? lo[2 * i + 1] : 0.0);
  }
  return U;
}

void apply1(Mps& m, int s, const std::vector<Cx>& U) {
  Site& S = m.site[s];
  Scratch sc;
  std::vector<Cx> in(2), out(2);
  for (int al = 0; al < S.ml; ++al)
    for (int be = 0; be < S.mr; ++be) {
      in[0] = S.at(al, 0, be); in[1] = S.at(al, 1, be);
      gate_mix(U, 2, in, out, sc);
      S.at(al, 0, be) = out[0]; S.at(al, 1, be) = out[1];
    }
}

// Split theta (rows (alpha,i) = 2a, columns = N) into Gamma_s', lambda_s' and the
// right factor Z_k (columns of V).  `lam_left` has a entries (lambda_{s-1}).
struct SplitOut {
  std::vector<Re> lam;  // k
  CMat Xg;              // Gamma_s' as (2a x k):  X / lambda_{s-1}
  CMat Zk;              // N x k : right singular vectors
};

SplitOut split(Mps& m, CMat& theta, const std::vector<Re>& lam_left, SplitStats& st) {
  const int M = theta.rows, N = theta.cols;
  Decomp d = decompose(theta, m.chi_max, m.eps);
  st = d.st;
  SplitOut o;
  const int k = d.k;
  o.lam.resize(k);
  for (int j = 0; j < k; ++j) mpfr_div(o.lam[j].v, d.sigma[j].v, d.nu.v, RN);
  o.Xg = CMat(M, k);
  o.Zk = CMat(N, k);
  for (int j = 0; j < k; ++j) {
    for (int r = 0; r < M; ++r) {
      const Re& l = lam_left[r / 2];
      mpfr_div(o.Xg.at(r, j).re.v, d.X.at(r, j).re.v, l.v, RN);
      mpfr_div(o.Xg.at(r, j).im.v, d.X.at(r, j).im.v, l.v, RN);
    }
    for (int r = 0; r < N; ++r) o.Zk.at(r, j) = d.Z.at(r, j);
  }
  return o;
}

void apply2(Mps& m, int s, const std::vector<Cx>& U) {
  Site& L = m.site[s];
  Site& Rt = m.site[s + 1];
  const int a = L.ml, b = L.mr, c = Rt.mr;
  Re one; mpfr_set_ui(one.v, 1, RN);
  // theta[(alpha,i), (j,gamma)], column index j*c + gamma
  CMat th(2 * a, 2 * c);
  const bool par = (size_t)a * b * c >= 4096;
  int nth = par ? omp_get_max_threads() : 1;
  std::vector<Scratch> scr(nth);
#pragma omp parallel for schedule(dynamic, 1) if (par)
  for (int al = 0; al < a; ++al) {
    Scratch& sc = scr[par ? omp_get_thread_num() : 0];
    std::vector<Cx> T(4), O(4);
    Cx lg;
    for (int ga = 0; ga < c; ++ga) {
      for (int ip = 0; ip < 2; ++ip)
        for (int jp = 0; jp < 2; ++jp) {
          Cx& acc = T[ip * 2 + jp];
          mpfr_set_ui(acc.re.v, 0, RN); mpfr_set_ui(acc.im.v, 0, RN);
          for (int be = 0; be < b; ++be) {
            // Gamma_s[al,ip,be] * lambda_s[be] * Gamma_{s+1}[be,jp,ga]
            Cx& x = L.at(al, ip, be);
            const Re& lb = lam_at(m, s, be, one);
            mpfr_mul(lg.re.v, x.re.v, lb.v, RN);
            mpfr_mul(lg.im.v, x.im.v, lb.v, RN);
            cfma(acc, lg, Rt.at(be, jp, ga), sc);
          }
        }
      gate_mix(U, 4, T, O, sc);
      Re w;
      mpfr_mul(w.v, lam_at(m, s - 1, al, one).v, lam_at(m, s + 1, ga, one).v, RN);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          Cx& dst = th.at(al * 2 + i, j * c + ga);
          mpfr_mul(dst.re.v, O[i * 2 + j].re.v, w.v, RN);
          mpfr_mul(dst.im.v, O[i * 2 + j].im.v, w.v, RN);
        }
    }
  }
  std::vector<Re> lam_left(a);
  for (int al = 0; al < a; ++al) lam_left[al] = lam_at(m, s - 1, al, one);
  SplitOut o = split(m, th, lam_left, m.last[0]);
  m.nsplits = 1;
  const int k = (int)o.lam.size();
  Site nL; nL.ml = a; nL.mr = k; nL.g.resize((size_t)a * 2 * k);
  for (int al = 0; al < a; ++al)
    for (int i = 0; i < 2; ++i)
      for (int nu = 0; nu < k; ++nu) nL.at(al, i, nu) = o.Xg.at(al * 2 + i, nu);
  Site nR; nR.ml = k; nR.mr = c; nR.g.resize((size_t)k * 2 * c);
  for (int nu = 0; nu < k; ++nu)
    for (int j = 0; j < 2; ++j)
      for (int ga = 0; ga < c; ++ga) {
        const Cx& z = o.Zk.at(j * c + ga, nu);
        Cx& dst = nR.at(nu, j, ga);
        const Re& lr = lam_at(m, s + 1, ga, one);
        mpfr_div(dst.re.v, z.re.v, lr.v, RN);
        mpfr_div(dst.im.v, z.im.v, lr.v, RN);
        mpfr_neg(dst.im.v, dst.im.v, RN);  // conj
      }
  m.site[s] = std::move(nL);
  m.site[s + 1] = std::move(nR);
  m.lam[s] = std::move(o.lam);
}

void apply3(Mps& m, int s, const std::vector<Cx>& U) {
  Site& S0 = m.site[s];
  Site& S1 = m.site[s + 1];
  Site& S2 = m.site[s + 2];
  const int a = S0.ml, b = S0.mr, c = S1.mr, d = S2.mr;
  Re one; mpfr_set_ui(one.v, 1, RN);
  // theta[(alpha,i), (j,k,delta)], column index (j*2+k)*d + delta
  CMat th(2 * a, 4 * d);
  const bool par = (size_t)a * (b * c + c * d) >= 4096;
  int nth = par ? omp_get_max_threads() : 1;
  std::vector<Scratch> scr(nth);
#pragma omp parallel for schedule(dynamic, 1) if (par)
  for (int al = 0; al < a; ++al) {
    Scratch& sc = scr[par ? omp_get_thread_num() : 0];
    // T1[ip][jp][ga] = sum_be Gamma0[al,ip,be] lam0[be] Gamma1[be,jp,ga] lam1[ga]
    std::vector<Cx> T1((size_t)4 * c);
    Cx lg;
    for (int ip = 0; ip < 2; ++ip)
      for (int jp = 0; jp < 2; ++jp)
        for (int ga = 0; ga < c; ++ga) {
          Cx& acc = T1[(ip * 2 + jp) * c + ga];
          for (int be = 0; be < b; ++be) {
            Cx& x = S0.at(al, ip, be);
            const Re& lb = lam_at(m, s, be, one);
            mpfr_mul(lg.re.v, x.re.v, lb.v, RN);
            mpfr_mul(lg.im.v, x.im.v, lb.v, RN);
            cfma(acc, lg, S1.at(be, jp, ga), sc);
          }
          const Re& lc = lam_at(m, s + 1, ga, one);
          mpfr_mul(acc.re.v, acc.re.v, lc.v, RN);
          mpfr_mul(acc.im.v, acc.im.v, lc.v, RN);
        }
    std::vector<Cx> T(8), O(8);
    for (int de = 0; de < d; ++de) {
      for (int ip = 0; ip < 2; ++ip)
        for (int jp = 0; jp < 2; ++jp)
          for (int kp = 0; kp < 2; ++kp) {
            Cx& acc = T[ip * 4 + jp * 2 + kp];
            mpfr_set_ui(acc.re.v, 0, RN); mpfr_set_ui(acc.im.v, 0, RN);
            for (int ga = 0; ga < c; ++ga) cfma(acc, T1[(ip * 2 + jp) * c + ga], S2.at(ga, kp, de), sc);
          }
      gate_mix(U, 8, T, O, sc);
      Re w;
      mpfr_mul(w.v, lam_at(m, s - 1, al, one).v, lam_at(m, s + 2, de, one).v, RN);
      for (int i = 0; i < 2; ++i)
        for (int jk = 0; jk < 4; ++jk) {
          Cx& dst = th.at(al * 2 + i, jk * d + de);
          mpfr_mul(dst.re.v, O[i * 4 + jk].re.v, w.v, RN);
          mpfr_mul(dst.im.v, O[i * 4 + jk].im.v, w.v, RN);
        }
    }
  }
  // split 1: (s | s+1 s+2)
  std::vector<Re> lam_left(a);
  for (int al = 0; al < a; ++al) lam_left[al] = lam_at(m, s - 1, al, one);
  SplitOut o1 = split(m, th, lam_left, m.last[0]);
  const int k1 = (int)o1.lam.size();
  // theta2[(nu,j), (k,delta)] = lambda_s'[nu] conj(Z1[(j,k,delta), nu])
  CMat th2(2 * k1, 2 * d);
  for (int nu = 0; nu < k1; ++nu)
    for (int j = 0; j < 2; ++j)
      for (int kk = 0; kk < 2; ++kk)
        for (int de = 0; de < d; ++de) {
          const Cx& z = o1.Zk.at((j * 2 + kk) * d + de, nu);
          Cx& dst = th2.at(nu * 2 + j, kk * d + de);
          mpfr_mul(dst.re.v, z.re.v, o1.lam[nu].v, RN);
          mpfr_mul(dst.im.v, z.im.v, o1.lam[nu].v, RN);
          mpfr_neg(dst.im.v, dst.im.v, RN);
        }
  SplitOut o2 = split(m, th2, o1.lam, m.last[1]);
  m.nsplits = 2;
  const int k2 = (int)o2.lam.size();
  Site n0; n0.ml = a; n0.mr = k1; n0.g.resize((size_t)a * 2 * k1);
  for (int al = 0; al < a; ++al)
    for (int i = 0; i < 2; ++i)
      for (int nu = 0; nu < k1; ++nu) n0.at(al, i, nu) = o1.Xg.at(al * 2 + i, nu);
  Site n1; n1.ml = k1; n1.mr = k2; n1.g.resize((size_t)k1 * 2 * k2);
  for (int nu = 0; nu < k1; ++nu)
    for (int j = 0; j < 2; ++j)
      for (int mu = 0; mu < k2; ++mu) n1.at(nu, j, mu) = o2.Xg.at(nu * 2 + j, mu);
  Site n2; n2.ml = k2; n2.mr = d; n2.g.resize((size_t)k2 * 2 * d);
  for (int mu = 0; mu < k2; ++mu)
    for (int kk = 0; kk < 2; ++kk)
      for (int de = 0; de < d; ++de) {
        const Cx& z = o2.Zk.at(kk * d + de, mu);
        Cx& dst = n2.at(mu, kk, de);
        const Re& lr = lam_at(m, s + 2, de, one);
        mpfr_div(dst.re.v, z.re.v, lr.v, RN);
        mpfr_div(dst.im.v, z.im.v, lr.v, RN);
        mpfr_neg(dst.im.v, dst.im.v, RN);
      }
  m.site[s] = std::move(n0);
  m.site[s + 1] = std::move(n1);
  m.site[s + 2] = std::move(n2);
  m.lam[s] = std::move(o1.lam);
  m.lam[s + 1] = std::move(o2.lam);
}

// ---------------------------------------------------------------- state vector
struct Sv {
  int n, prec;
  CVec psi;
};

}  // namespace

// ====================================================================== C ABI
extern "C" {

// MPS oracle in Gamma-lambda form, initialised to |0...0> (all m_s = 1).
void* omps_create(int n, int chi_max, double eps, int prec_bits) {
  if (n < 1 || chi_max < 1 || !(eps >= 0) || prec_bits < 64) return nullptr;
  g_prec = prec_bits;
  Mps* m = new Mps();
  m->n = n; m->chi_max = chi_max; m->eps = eps; m->prec = prec_bits;
  m->site.resize(n);
  for (int s = 0; s < n; ++s) {
    m->site[s].g.resize(2);
    mpfr_set_ui(m->site[s].g[0].re.v, 1, RN);
  }
  m->lam.resize(n > 1 ? n - 1 : 0);
  for (int s = 0; s + 1 < n; ++s) {
    m->lam[s].resize(1);
    mpfr_set_ui(m->lam[s][0].v, 1, RN);
  }
  return m;
}

void omps_destroy(void* h) {
  if (!h) return;
  Mps* m = (Mps*)h;
  g_prec = m->prec;
  delete m;
}

void omps_set_max_sweeps(int s) { g_max_sweeps = s; }

// Change the truncation parameters of a handle for the gates that follow.
int omps_set_trunc(void* h, int chi_max, double eps) {
  Mps* m = (Mps*)h;
  if (!m || chi_max < 1 || !(eps >= 0)) return -1;
  m->chi_max = chi_max;
  m->eps = eps;
  return 0;
}

// Apply a k-site gate (k = 1, 2, 3) on sites first..first+k-1.  u_hi/u_lo hold
// 2*4^k doubles, row-major, complex interleaved; u_lo may be NULL.
// Returns 0, or -1 on bad arguments, -5 if a Jacobi iteration did not converge.
int omps_apply(void* h, int first, int k, const double* u_hi, const double* u_lo) {
  Mps* m = (Mps*)h;
  if (!m || !u_hi || k < 1 || k > 3 || first < 0 || first + k > m->n) return -1;
  g_prec = m->prec;
  std::vector<Cx> U = load_gate(k, u_hi, u_lo);
  m->nsplits = 0;
  if (k == 1) apply1(*m, first, U);
  else if (k == 2) apply2(*m, first, U);
  else apply3(*m, first, U);
  for (int i = 0; i < m->nsplits; ++i)
    if (!m->last[i].converged) return -5;
  return 0;
}

int omps_bond_dim(void* h, int bond) {
  Mps* m = (Mps*)h;
  if (!m || bond < 0 || bond >= m->n - 1) return -1;
  return (int)m->lam[bond].size();
}

// Schmidt values of bond `bond` (descending) as (hi, lo) pairs; returns m or -1.
int omps_schmidt(void* h, int bond, double* hi, double* lo, int cap) {
  Mps* m = (Mps*)h;
  if (!m || bond < 0 || bond >= m->n - 1) return -1;
  g_prec = m->prec;
  int mm = (int)m->lam[bond].size();
  for (int j = 0; j < mm && j < cap; ++j) get_d2(m->lam[bond][j].v, &hi[j], &lo[j]);
  return mm;
}

// Amplitude <b_0 ... b_{n-1}|Psi> from Eq. (1):
// Gamma_0[b0] lambda_0 Gamma_1[b1] lambda_1 ... Gamma_{n-1}[b_{n-1}].
// out = {re_hi, re_lo, im_hi, im_lo}.
int omps_amplitude(void* h, const unsigned char* bits, double* out) {
  Mps* m = (Mps*)h;
  if (!m || !bits || !out) return -1;
  g_prec = m->prec;
  Scratch sc;
  CVec v(1);
  mpfr_set_ui(v[0].re.v, 1, RN);
  for (int s = 0; s < m->n; ++s) {
    Site& S = m->site[s];
    const int bs = bits[s] ? 1 : 0;
    CVec w(S.mr);
    for (int be = 0; be < S.mr; ++be)
      for (int al = 0; al < S.ml; ++al) cfma(w[be], v[al], S.at(al, bs, be), sc);
    if (s < m->n - 1)
      for (int be = 0; be < S.mr; ++be) {
        mpfr_mul(w[be].re.v, w[be].re.v, m->lam[s][be].v, RN);
        mpfr_mul(w[be].im.v, w[be].im.v, m->lam[s][be].v, RN);
      }
    v = std::move(w);
  }
  get_d2(v[0].re.v, &out[0], &out[1]);
  get_d2(v[0].im.v, &out[2], &out[3]);
  return 0;
}

// Diagnostics of the last gate: per split 9 doubles
// {W_hi, W_lo, w_hi, w_lo, k, sweeps, gap, epsdist, rank}; returns the number of splits.
int omps_last_stats(void* h, double* out) {
  Mps* m = (Mps*)h;
  if (!m || !out) return -1;
  for (int i = 0; i < m->nsplits; ++i) {
    const SplitStats& s = m->last[i];
    double* o = out + 9 * i;
    o[0] = s.W_hi; o[1] = s.W_lo; o[2] = s.w_hi; o[3] = s.w_lo;
    o[4] = s.k; o[5] = s.sweeps; o[6] = s.gap; o[7] = s.epsdist; o[8] = s.rank;
  }
  return m->nsplits;
}

// Replace the state by an MPS given in the (B, lambda) gauge, B_s = Gamma_s lambda_s:
// dims[s] = m_s for s = 0..n-2; B_s is (m_{s-1} x 2 x m_s) complex, row-major
// [alpha][i][beta], (hi, lo) pairs; lambda_s has m_s entries.  The oracle stores
// Gamma_s = B_s / lambda_s.  lam_lo / b_lo may be NULL.
int omps_load(void* h, const int* dims, const double* const* b_hi, const double* const* b_lo,
              const double* const* lam_hi, const double* const* lam_lo) {
  Mps* m = (Mps*)h;
  if (!m || (m->n > 1 && !dims)) return -1;
  g_prec = m->prec;
  const int n = m->n;
  std::vector<int> full(n + 1, 1);
  for (int s = 0; s + 1 < n; ++s) full[s + 1] = dims[s];
  for (int s = 0; s + 1 < n; ++s) {
    m->lam[s].assign(dims[s], Re());
    for (int j = 0; j < dims[s]; ++j)
      set_d2(m->lam[s][j].v, lam_hi[s][j], lam_lo ? lam_lo[s][j] : 0.0);
  }
  Re one; mpfr_set_ui(one.v, 1, RN);
  for (int s = 0; s < n; ++s) {
    Site S; S.ml = full[s]; S.mr = full[s + 1];
    S.g.resize((size_t)S.ml * 2 * S.mr);
    for (size_t e = 0; e < S.g.size(); ++e) {
      const int be = (int)(e % S.mr);
      set_d2(S.g[e].re.v, b_hi[s][2 * e], b_lo ? b_lo[s][2 * e] : 0.0);
      set_d2(S.g[e].im.v, b_hi[s][2 * e + 1], b_lo ? b_lo[s][2 * e + 1] : 0.0);
      const Re& l = lam_at(*m, s, be, one);
      mpfr_div(S.g[e].re.v, S.g[e].re.v, l.v, RN);
      mpfr_div(S.g[e].im.v, S.g[e].im.v, l.v, RN);
    }
    m->site[s] = std::move(S);
  }
  return 0;
}

// Jacobi SVD of a general complex M x N matrix (column-major, complex interleaved,
// (hi, lo) pairs; a_lo may be NULL).  Outputs (hi, lo) pairs: sigma (N, descending),
// V (N x N, columns permuted to match sigma), W = A V (M x N, same permutation).
// Returns the number of sweeps, or -5 when not converged.
int osvd(int M, int N, const double* a_hi, const double* a_lo, int prec,
         double* sig_hi, double* sig_lo, double* v_hi, double* v_lo, double* w_hi, double* w_lo) {
  if (M < 1 || N < 1 || !a_hi) return -1;
  g_prec = prec;
  CMat A(M, N), V;
  for (size_t e = 0; e < (size_t)M * N; ++e) {
    set_d2(A.a[e].re.v, a_hi[2 * e], a_lo ? a_lo[2 * e] : 0.0);
    set_d2(A.a[e].im.v, a_hi[2 * e + 1], a_lo ? a_lo[2 * e + 1] : 0.0);
  }
  SvdResult r = jacobi_svd(A, V);
  std::vector<Re> sig;
  column_norms(A, sig);
  std::vector<int> order(N);
  for (int j = 0; j < N; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return mpfr_cmp(sig[x].v, sig[y].v) > 0; });
  for (int j = 0; j < N; ++j) {
    const int c = order[j];
    if (sig_hi) get_d2(sig[c].v, &sig_hi[j], &sig_lo[j]);
    for (int r2 = 0; r2 < N && v_hi; ++r2) {
      size_t o = 2 * ((size_t)j * N + r2);
      get_d2(V.at(r2, c).re.v, &v_hi[o], &v_lo[o]);
      get_d2(V.at(r2, c).im.v, &v_hi[o + 1], &v_lo[o + 1]);
    }
    for (int r2 = 0; r2 < M && w_hi; ++r2) {
      size_t o = 2 * ((size_t)j * M + r2);
      get_d2(A.at(r2, c).re.v, &w_hi[o], &w_lo[o]);
      get_d2(A.at(r2, c).im.v, &w_hi[o + 1], &w_lo[o + 1]);
    }
  }
  return r.converged ? r.sweeps : -5;
}

// Reduced density operator rho = Tr_{other qubits} |Psi><Psi| of the listed qubits
// (Section 3.2: RDO(list); RDO_block(a, b) is the list a..b), straight from the
// definition: |Psi><Psi| of Eq. (1) is contracted site by site from the left,
//   env[(I, I')][beta][beta'] = sum over all indices left of the cut, except the
//                               listed ones (I, I'), of c(.., beta) conj(c(.., beta')),
// with the site matrices M_s[i] = Q_s[i] V_s (V_{n-1} = [1]).  A listed site opens a
// pair (i, i'), any other site is traced (i = i').  No canonical form is assumed.
// out: 2^L x 2^L, row-major, 4 doubles per entry (re_hi, re_lo, im_hi, im_lo); the
// row index is sum_t i_{q[t]} 2^{L-1-t} for the qubits in the order given.
int omps_rdo(void* h, int L, const int* q, double* out) {
  Mps* m = (Mps*)h;
  if (!m || !q || !out || L < 1 || L > 10) return -1;
  const int n = m->n;
  std::vector<char> listed(n, 0);
  for (int t = 0; t < L; ++t) {
    if (q[t] < 0 || q[t] >= n || listed[q[t]]) return -1;
    listed[q[t]] = 1;
  }
  g_prec = m->prec;
  Re one; mpfr_set_ui(one.v, 1, RN);
  int l = 0, mcur = 1;  // listed qubits opened so far, current bond dim
  std::vector<CVec> env(1, CVec(1));
  mpfr_set_ui(env[0][0].re.v, 1, RN);
  for (int s = 0; s < n; ++s) {
    Site& S = m->site[s];
    const int ml = S.ml, mr = S.mr;
    // M_s[i] = Q_s[i] V_s
    CVec M((size_t)ml * 2 * mr);
    for (int al = 0; al < ml; ++al)
      for (int i = 0; i < 2; ++i)
        for (int be = 0; be < mr; ++be) {
          const Re& lv = lam_at(*m, s, be, one);
          Cx& x = M[((size_t)al * 2 + i) * mr + be];
          mpfr_mul(x.re.v, S.at(al, i, be).re.v, lv.v, RN);
          mpfr_mul(x.im.v, S.at(al, i, be).im.v, lv.v, RN);
        }
    auto Mat = [&](int al, int i, int be) -> const Cx& { return M[((size_t)al * 2 + i) * mr + be]; };
    const int D = (int)env.size();
    const bool open = listed[s] != 0;
    const int Dn = open ? 4 * D : D;
    std::vector<CVec> nenv(Dn, CVec((size_t)mr * mr));
    // F[d][i][al'][be] = sum_al env[d][al][al'] M[al][i][be]
    std::vector<CVec> F(D, CVec((size_t)2 * ml * mr));
#pragma omp parallel for collapse(2) schedule(dynamic, 1) if (D * ml * mr > 256)
    for (int d = 0; d < D; ++d)
      for (int ap = 0; ap < ml; ++ap) {
        Scratch sc;
        for (int i = 0; i < 2; ++i)
          for (int be = 0; be < mr; ++be) {
            Cx& f = F[d][((size_t)i * ml + ap) * mr + be];
            for (int al = 0; al < ml; ++al) cfma(f, env[d][(size_t)al * mcur + ap], Mat(al, i, be), sc);
          }
      }
    // env'[..][be][be'] = sum_al' F[d][i][al'][be] conj(M[al'][i'][be'])
#pragma omp parallel for collapse(2) schedule(dynamic, 1) if (D * mr * mr > 256)
    for (int d = 0; d < D; ++d)
      for (int be = 0; be < mr; ++be) {
        Scratch sc;
        const int I = d >> l, Ip = d & ((1 << l) - 1);
        for (int bp = 0; bp < mr; ++bp)
          for (int i = 0; i < 2; ++i)
            for (int ip = 0; ip < 2; ++ip) {
              if (!open && ip != i) continue;
              const int dn = open ? ((2 * I + i) << (l + 1)) + (2 * Ip + ip) : d;
              Cx& e = nenv[dn][(size_t)be * mr + bp];
              for (int ap = 0; ap < ml; ++ap) cfma_cj(e, F[d][((size_t)i * ml + ap) * mr + be], Mat(ap, ip, bp), sc);
            }
      }
    env = std::move(nenv);
    mcur = mr;
    if (open) ++l;
  }
  // sorted order of the listed qubits -> the requested order
  std::vector<int> sorted;
  for (int s = 0; s < n; ++s)
    if (listed[s]) sorted.push_back(s);
  std::vector<int> pos(L);  // bit position (from the MSB) of q[t] in the sorted index
  for (int t = 0; t < L; ++t)
    pos[t] = (int)(std::find(sorted.begin(), sorted.end(), q[t]) - sorted.begin());
  const int dim = 1 << L;
  for (int r = 0; r < dim; ++r)
    for (int c = 0; c < dim; ++c) {
      int rs = 0, cs = 0;
      for (int t = 0; t < L; ++t) {
        rs |= ((r >> (L - 1 - t)) & 1) << (L - 1 - pos[t]);
        cs |= ((c >> (L - 1 - t)) & 1) << (L - 1 - pos[t]);
      }
      const Cx& v = env[((size_t)rs << L) + cs][0];
      double* o = out + 4 * ((size_t)r * dim + c);
      get_d2(v.re.v, &o[0], &o[1]);
      get_d2(v.im.v, &o[2], &o[3]);
    }
  return 0;
}

// Dense state vector of n qubits at `prec` bits, |0...0>.  Basis index
// sum_q i_q 2^{n-1-q}: qubit 0 is the most significant bit.
void* osv_create(int n, int prec_bits) {
  if (n < 1 || n > 24) return nullptr;
  g_prec = prec_bits;
  Sv* v = new Sv();
  v->n = n; v->prec = prec_bits;
  v->psi.resize((size_t)1 << n);
  mpfr_set_ui(v->psi[0].re.v, 1, RN);
  return v;
}

void osv_destroy(void* h) {
  if (!h) return;
  Sv* v = (Sv*)h;
  g_prec = v->prec;
  delete v;
}

// Apply a gate on the listed qubits (qubits[0] = most significant bit of the gate
// index); any qubits, adjacent or not.
int osv_apply(void* h, int nq, const int* qubits, const double* u_hi, const double* u_lo) {
  Sv* v = (Sv*)h;
  if (!v || nq < 1 || nq > 3 || !qubits || !u_hi) return -1;
  g_prec = v->prec;
  const int n = v->n, d = 1 << nq;
  std::vector<Cx> U = load_gate(nq, u_hi, u_lo);
  size_t mask = 0;
  std::vector<size_t> bit(nq);
  for (int t = 0; t < nq; ++t) {
    if (qubits[t] < 0 || qubits[t] >= n) return -1;
    bit[t] = (size_t)1 << (n - 1 - qubits[t]);
    mask |= bit[t];
  }
  Scratch sc;
  std::vector<Cx> in(d), out(d);
  std::vector<size_t> idx(d);
  for (size_t base = 0; base < v->psi.size(); ++base) {
    if (base & mask) continue;
    for (int r = 0; r < d; ++r) {
      size_t x = base;
      for (int t = 0; t < nq; ++t)
        if ((r >> (nq - 1 - t)) & 1) x |= bit[t];
      idx[r] = x;
      in[r] = v->psi[x];
    }
    gate_mix(U, d, in, out, sc);
    for (int r = 0; r < d; ++r) v->psi[idx[r]] = out[r];
  }
  return 0;
}

// All 2^n amplitudes as {re_hi, re_lo, im_hi, im_lo} per index.
int osv_amplitudes(void* h, double* out) {
  Sv* v = (Sv*)h;
  if (!v || !out) return -1;
  g_prec = v->prec;
  for (size_t i = 0; i < v->psi.size(); ++i) {
    get_d2(v->psi[i].re.v, &out[4 * i], &out[4 * i + 1]);
    get_d2(v->psi[i].im.v, &out[4 * i + 2], &out[4 * i + 3]);
  }
  return 0;
}

int oracle_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
