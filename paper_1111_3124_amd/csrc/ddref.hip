// Double-double refinement of a converged FP64 one-sided Jacobi, by simultaneous
// first-order corrections (gfx950).
//
// On entry (after the dd promotion and Newton-Schulz steps) V is unitary to dd
// precision and W = theta_w V (dd; theta_w^H V for a wide theta) has nearly orthogonal columns: the off-diagonal
// Gram entries g_pq are ~2^-53 sqrt(g_pp g_qq) (the FP64 Jacobi's stopping point).
// All pairs are then corrected at once, as in the matrix-multiplication based SVD
// refinement of Ogita and Aishima (J. Comput. Appl. Math. 369, 2020), in its
// one-sided form:
//   G = W^H W                          (dd accumulation; diagonal kept in dd)
//   E_pq = g_pq / (g_qq - g_pp), E_qp = -conj(E_pq), E_pp = 0      (E anti-Hermitian)
//   F = E + E^2 / 2                    (I + F is unitary to O(|E|^4))
//   W <- W + W_hi F,  V <- V + V_hi F  (binary64 products, dd sums)
// The first-order term removes g_pq exactly; what is left is of second order, so
// each pass squares the relative off-diagonal size: two passes take the FP64 level
// below the dd tolerance.  The binary64 products suffice because F is tiny: their
// rounding is 2^-53 |F| relative to W.  sigma^2 is taken from the updated columns.
//
// A pair whose E_pq would exceed 1e-8 (a relative gap below ~1e-5: near-degenerate
// singular values) voids the pass for that task (nothing is updated) and the task
// goes to the pairwise dd Jacobi polish instead.
//
// Passes are numbered per task; pass q writes its outcome to flags[q % 3] (0: every
// pair at the convergence level, |1: some pair above it, |2: void) and clears
// flags[(q + 1) % 3] for the next one.  Pass q > 0 runs only if pass q - 1 ended
// with exactly 1 (corrected, not yet converged), so consecutive passes can be
// queued together: those after a converged or void pass leave everything untouched.
#include "dd.h"
#include "ddgemm.h"
#include "ddref.h"
#include "gemm.h"

namespace mpsk {

namespace {
constexpr double kMaxE = 1e-8;  // larger corrections are left to the pairwise polish
}

// G = W^H W on the upper tiles: the diagonal goes to sig2 (dd), the rest to aux1
// (binary64, column-major, upper triangle read by k_ref_e)
struct WGramOp {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = false;
  const Task2* t;
  __device__ cdd a(int row, int kk) const { return dd::cconj(ldc(t->thw, t->thw_lo, (long)row * t->JM + kk)); }
  __device__ cdd b(int kk, int col) const { return ldc(t->thw, t->thw_lo, (long)col * t->JM + kk); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const int N = t->N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r >= N || c >= N) continue;
        if (r == c) {
          t->sig2[r] = v[i][j].re.hi;
          t->sig2_lo[r] = v[i][j].re.lo;
        } else {
          t->aux1[(long)c * N + r] = make_double2(v[i][j].re.hi, v[i][j].im.hi);
        }
      }
  }
};

// pass q > 0 follows a pass that corrected without converging
__device__ __forceinline__ bool ref_skip(const Task2& T, int pass) {
  return pass > 0 && T.flags[(pass + 2) % 3] != 1;
}

__global__ __launch_bounds__(256) void k_ref_gram(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->N || tn >= t->N || tm > tn) return;  // upper tiles (and the diagonal ones)
  if (ref_skip(*t, ents[blockIdx.z].sweep)) return;
  if (tm == 0 && tn == 0 && threadIdx.x == 0) t->flags[(ents[blockIdx.z].sweep + 1) % 3] = 0;
  WGramOp op{t};
  ddgemm_tile(op, t->N, t->N, t->JM, tm, tn);
}

// E from G; flags[pass % 3] |= 1 while some pair is above the convergence level,
// |= 2 if some correction is too large for a first-order step
__global__ __launch_bounds__(256) void k_ref_e(Task2* tasks, const Ent* ents, double tol_mult) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int pass = ents[blockIdx.y].sweep;
  if (ref_skip(T, pass)) return;  // the whole block: the flag is the task's
  const int N = T.N, M = T.JM;
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-101;
  const double rtol = sqrt(tol / (double)(N > 1 ? N : 1));
  const double ztol = *T.fro2 * 0x1p-192;
  int code = 0;
  const long nn = (long)N * N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
    const int p = (int)(e % N), q = (int)(e / N);
    if (p > q) continue;  // (q, p) is written with (p, q)
    if (p == q) {
      T.aux1[e] = cmk(0.0, 0.0);
      continue;
    }
    const double2 g = T.aux1[e];
    const ddr al = {T.sig2[p], T.sig2_lo[p]}, be = {T.sig2[q], T.sig2_lo[q]};
    double2 ep = cmk(0.0, 0.0);
    if (al.hi > ztol && be.hi > ztol) {
      const double g2 = g.x * g.x + g.y * g.y;
      if (g2 > rtol * rtol * al.hi * be.hi) code |= 1;
      const double d = dd::sub(be, al).hi;
      if (g2 == 0.0) {
        // already orthogonal
      } else if (sqrt(g2) > kMaxE * fabs(d)) {
        code |= 2;
      } else {
        const double id = 1.0 / d;
        ep = cmk(g.x * id, g.y * id);
      }
    }
    T.aux1[e] = ep;                                        // E_pq
    T.aux1[(long)p * N + q] = cmk(-ep.x, ep.y);            // E_qp = -conj(E_pq)
  }
  // one flag update per block (the same word is shared by all of the task's blocks)
  const int c1 = __syncthreads_or(code & 1), c2 = __syncthreads_or(code & 2);
  if (threadIdx.x == 0 && (c1 || c2)) atomicOr(&T.flags[pass % 3], (c1 ? 1 : 0) | (c2 ? 2 : 0));
}

__device__ __forceinline__ bool ref_void(const Task2& T, int pass) {
  return ref_skip(T, pass) || (T.flags[pass % 3] & 2) != 0;
}

// F = E + E^2 / 2 into aux2
struct RefSqOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  __device__ double2 a(int row, int kk) const { return t->aux1[(long)kk * t->N + row]; }
  __device__ double2 b(int kk, int col) const { return t->aux1[(long)col * t->N + kk]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int N = t->N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r < N && c < N) {
          const long o = (long)c * N + r;
          t->aux2[o] = cadd(t->aux1[o], cscale(acc[i][j], 0.5));
        }
      }
  }
};

__global__ __launch_bounds__(256) void k_ref_sq(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->N || tn >= t->N || ref_void(*t, ents[blockIdx.z].sweep)) return;
  RefSqOp op{t};
  cgemm_tile(op, t->N, t->N, t->N, tm, tn);
}

// X_hi F for X = W (M x N, into aux3) and X = V (N x N, into aux1: E is no longer
// needed once F is formed); blockIdx.x tiles W's rows first, then V's
struct RefMulOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const double2* X;
  const double2* F;
  double2* out;
  int rows, N;
  __device__ double2 a(int row, int kk) const { return X[(long)kk * rows + row]; }
  __device__ double2 b(int kk, int col) const { return F[(long)col * N + kk]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r < rows && c < N) out[(long)c * rows + r] = acc[i][j];
      }
  }
};

__global__ __launch_bounds__(256) void k_ref_mul(Task2* tasks, const Ent* ents, int wtiles) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  if (ref_void(*t, ents[blockIdx.z].sweep)) return;
  const bool isw = (int)blockIdx.x < wtiles;
  const int tm = (isw ? blockIdx.x : blockIdx.x - wtiles) * 64, tn = blockIdx.y * 64;
  const int rows = isw ? t->JM : t->N;
  if (tm >= rows || tn >= t->N) return;
  RefMulOp op{isw ? t->thw : t->V, t->aux2, isw ? t->aux3 : t->aux1, rows, t->N};
  cgemm_tile(op, rows, t->N, t->N, tm, tn);
}

// W += aux3, V += aux1 (dd sums), sigma^2 = |W column|^2 in dd: a block per column
__global__ __launch_bounds__(256) void k_ref_add(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int c = blockIdx.x, M = T.JM, N = T.N;
  if (c >= N || ref_void(T, ents[blockIdx.y].sweep)) return;
  const int tid = threadIdx.x;
  cacc s = cacc0();
  for (int r = tid; r < M; r += 256) {
    const long o = (long)c * M + r;
    cdd w = ldc(T.thw, T.thw_lo, o);
    const double2 d = T.aux3[o];
    w.re = dd::add_d(w.re, d.x);
    w.im = dd::add_d(w.im, d.y);
    stc(T.thw, T.thw_lo, o, w);
    dd::cacc_fmac(s, w, w);
  }
  for (int r = tid; r < N; r += 256) {
    const long o = (long)c * N + r;
    cdd v = ldc(T.V, T.V_lo, o);
    const double2 d = T.aux1[o];
    v.re = dd::add_d(v.re, d.x);
    v.im = dd::add_d(v.im, d.y);
    stc(T.V, T.V_lo, o, v);
  }
  __shared__ ddr red[256];
  red[tid] = dd::norm(s.re);
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] = dd::add(red[tid], red[tid + k]);
    __syncthreads();
  }
  if (tid == 0) {
    T.sig2[c] = red[0].hi;
    T.sig2_lo[c] = red[0].lo;
  }
}

__global__ __launch_bounds__(64) void k_flags_clear(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.x].slot];
  if (threadIdx.x < 3) T.flags[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_ddref_pass(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, double tol_mult,
                             hipStream_t st) {
  const int t32 = (maxN + 31) / 32, t64 = (maxN + 63) / 64;
  hipLaunchKernelGGL(k_ref_gram, dim3(t32, t32, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  long nn = (long)maxN * maxN;
  int ge = (int)std::min<long>((nn + 255) / 256, 1024);
  hipLaunchKernelGGL(k_ref_e, dim3(ge, nent), dim3(256), 0, st, d_tasks, d_ents, tol_mult);
  MPS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ref_sq, dim3(t64, t64, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  const int wt = (maxM + 63) / 64;
  hipLaunchKernelGGL(k_ref_mul, dim3(wt + t64, t64, nent), dim3(256), 0, st, d_tasks, d_ents, wt);
  MPS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ref_add, dim3(maxN, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_flags_clear(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st) {
  hipLaunchKernelGGL(k_flags_clear, dim3(nent), dim3(64), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
