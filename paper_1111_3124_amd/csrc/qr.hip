// QR preconditioning of wide thetas (gfx950), FP64 and double-double.
//
// When theta_w has fewer rows than columns (M < Nt: the left half of a chain, where
// bond dimensions grow to the right, and the first split of a three-site gate), a
// one-sided Jacobi on its Nt columns has to drive Nt - M of them to zero, which it
// does only linearly.  Instead, as in the QR-preconditioned one-sided Jacobi SVD
// (Drmac and Veselic, SIAM J. Matrix Anal. Appl. 29, 2008):
//   theta_w^H = Q R            Householder QR: Q (Nt x M) orthonormal columns, R (M x M)
//   theta_w   = R^H Q^H        one-sided Jacobi on the M columns of R^H: R^H V_R = X Sigma
//   Z         = Q V_R          right singular vectors of theta_w, formed for the kept
//                              columns only, after the truncation
// The Jacobi sweeps, the dd refinement and the truncation see the square R^H; the
// split (B_{s+1}' = Z_k^H, B_s' = theta Z_k / nu) reads Z_k.
//
// The QR is one workgroup per task: column j's reflector (LAPACK's zlarfg
// convention: H = I - tau v v^H, v_j = 1, H^H x = beta e_1 with beta real) is
// formed by one wave, then the 16 waves update the trailing columns, a group of
// columns per wave at a time (lanes stride the rows, each dot product is a wave
// butterfly, whose result is bit-identical on every lane).  Q is then accumulated
// in place, last reflector first (as LAPACK's zung2r).
#include "dd.h"
#include "ddgemm.h"
#include "gemm.h"
#include "qr.h"

namespace mpsk {

namespace {

constexpr int kQrThreads = 1024;
constexpr int kQrWaves = kQrThreads / 64;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ ddr wave_sum_dd(ddr x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const ddr y = {__shfl_xor(x.hi, o, 64), __shfl_xor(x.lo, o, 64)};
    x = dd::add(x, y);  // dd addition is commutative bit for bit: all lanes agree
  }
  return x;
}

}  // namespace

// ------------------------------------------------------------------ FP64
// Column j's reflector from the (already updated) column: the norm of rows > j is a
// wave butterfly, so every lane of the calling wave forms the same beta, tau and
// scale; the wave scales the column into v (v_j = 1 implied, beta stored at A(j, j)).
__device__ __forceinline__ double2 make_reflector(double2* aj, int j, int Nt, int lane) {
  double s = 0.0;
  for (int r = j + 1 + lane; r < Nt; r += 64) {
    const double2 x = aj[r];
    s = fma(x.x, x.x, fma(x.y, x.y, s));
  }
  s = wave_sum(s);
  const double2 al = aj[j];
  if (!(s > 0.0 || al.y != 0.0)) return cmk(0.0, 0.0);  // H = I
  const double nrm = sqrt(al.x * al.x + al.y * al.y + s);
  const double be = al.x >= 0.0 ? -nrm : nrm;
  const double2 dz = cmk(al.x - be, al.y);  // alpha - beta
  const double id = 1.0 / (dz.x * dz.x + dz.y * dz.y);
  const double2 sc = cmk(dz.x * id, -dz.y * id);
  for (int r = j + 1 + lane; r < Nt; r += 64) aj[r] = cmul(aj[r], sc);
  if (lane == 0) aj[j] = cmk(be, 0.0);
  return cmk((be - al.x) / be, -al.y / be);
}

// A[i0.., c] -= (mult * v^H A[i0.., c]) v for the wave's columns c = c0 + 16 q (q < nc),
// v = column i0 of A with v_i0 = 1: up to kCB columns per pass, so that their loads
// and butterflies overlap.
constexpr int kCB = 4;
__device__ __forceinline__ void apply_reflector_cols(double2* A, int Nt, int i0, double2 mult, int c0, int nc,
                                                     int lane) {
  const double2* v = A + (long)i0 * Nt;
  double2 dot[kCB];
#pragma unroll
  for (int q = 0; q < kCB; ++q) dot[q] = cmk(0.0, 0.0);
  for (int r = i0 + lane; r < Nt; r += 64) {
    const double2 vr = r == i0 ? cmk(1.0, 0.0) : v[r];
#pragma unroll
    for (int q = 0; q < kCB; ++q)
      if (q < nc) dot[q] = cfmac(vr, A[(long)(c0 + kQrWaves * q) * Nt + r], dot[q]);
  }
  double2 f[kCB];
#pragma unroll
  for (int q = 0; q < kCB; ++q) {
    dot[q].x = wave_sum(dot[q].x);
    dot[q].y = wave_sum(dot[q].y);
    f[q] = cmul(mult, dot[q]);
  }
  for (int r = i0 + lane; r < Nt; r += 64) {
    const double2 vr = r == i0 ? cmk(1.0, 0.0) : v[r];
#pragma unroll
    for (int q = 0; q < kCB; ++q)
      if (q < nc) {
        double2* p = A + (long)(c0 + kQrWaves * q) * Nt + r;
        *p = csub(*p, cmul(vr, f[q]));
      }
  }
}

// Q's column i from its reflector once H_i has been applied to the later columns:
// (I - tau_i v v^H) e_i = e_i - tau_i v
__device__ __forceinline__ void finish_q_col(double2* ai, int i, int Nt, double2 ti, int lane) {
  for (int r = lane; r < Nt; r += 64) {
    if (r < i)
      ai[r] = cmk(0.0, 0.0);
    else if (r == i)
      ai[r] = cmk(1.0 - ti.x, -ti.y);
    else
      ai[r] = cmul(cmk(-ti.x, -ti.y), ai[r]);
  }
}

// One barrier per Householder step: the wave that updates column j+1 (wave 0, whose
// first column it is) forms reflector j+1 right after, while the other waves still
// update theirs.
__global__ __launch_bounds__(kQrThreads) void k_qr(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.x].slot];
  const int M = T.M, Nt = T.Nt;
  double2* __restrict__ A = T.Qh;  // Nt x M, column-major
  double2* __restrict__ tau = T.tau;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double2 s_tau[2];  // double-buffered by step parity

  // A = theta_w^H
  for (long e = tid; e < (long)M * Nt; e += kQrThreads) {
    const int m = (int)(e % M), n = (int)(e / M);
    A[(long)m * Nt + n] = cconj(T.thw[e]);
  }
  __syncthreads();
  if (wave == 0) {
    const double2 t0 = make_reflector(A, 0, Nt, lane);
    if (lane == 0) {
      tau[0] = t0;
      s_tau[0] = t0;
    }
  }
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    const double2 tj = s_tau[j & 1];
    const bool act = tj.x != 0.0 || tj.y != 0.0;
    const double2 ctj = cconj(tj);  // A <- H^H A = A - conj(tau) v (v^H A)
    int c0 = j + 1 + wave;
    if (wave == 0 && j + 1 < M) {
      // first the column of the next reflector, then that reflector
      if (act) apply_reflector_cols(A, Nt, j, ctj, c0, min(kCB, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
      __threadfence_block();  // lanes now read rows other lanes of this wave wrote
      const double2 tn = make_reflector(A + (long)(j + 1) * Nt, j + 1, Nt, lane);
      if (lane == 0) {
        tau[j + 1] = tn;
        s_tau[(j + 1) & 1] = tn;
      }
      c0 += kQrWaves * kCB;
    }
    if (act)
      for (; c0 < M; c0 += kQrWaves * kCB)
        apply_reflector_cols(A, Nt, j, ctj, c0, min(kCB, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
    __syncthreads();
  }

  // the Jacobi matrix R^H (M x M, lower triangular)
  for (long e = tid; e < (long)M * M; e += kQrThreads) {
    const int r = (int)(e % M), c = (int)(e / M);
    T.thw[e] = r >= c ? cconj(A[(long)r * Nt + c]) : cmk(0.0, 0.0);
  }
  __syncthreads();

  // Q = H_0 H_1 ... H_{M-1} [I; 0] in place, last reflector first; column i+1 is
  // finished by wave 0 in step i, before it applies H_i to it
  for (int i = M - 1; i >= 0; --i) {
    const double2 ti = tau[i];
    const bool act = ti.x != 0.0 || ti.y != 0.0;
    int c0 = i + 1 + wave;
    if (wave == 0 && i + 1 < M) {
      finish_q_col(A + (long)(i + 1) * Nt, i + 1, Nt, tau[i + 1], lane);
      __threadfence_block();
      if (act) apply_reflector_cols(A, Nt, i, ti, c0, min(kCB, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
      c0 += kQrWaves * kCB;
    }
    if (act)
      for (; c0 < M; c0 += kQrWaves * kCB)
        apply_reflector_cols(A, Nt, i, ti, c0, min(kCB, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
    __syncthreads();
  }
  if (wave == 0) finish_q_col(A, 0, Nt, tau[0], lane);
}

// Z[:, nu] = Q V_R[:, perm[nu]] for the kept columns nu < k
struct ZformOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  int k;
  __device__ double2 a(int row, int kk) const { return t->Qh[(long)kk * t->Nt + row]; }
  __device__ double2 b(int kk, int col) const { return t->V[(long)t->perm[col] * t->N + kk]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + i;
      if (r >= t->Nt) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = c0 + j;
        if (c < k) t->Z[(long)c * t->Nt + r] = acc[i][j];
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_zform(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int k = *t->dim_out;
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->Nt || tn >= k) return;
  ZformOp op{t, k};
  cgemm_tile(op, t->Nt, k, t->N, tm, tn);
}

// ------------------------------------------------------------------ double-double
// The same factorisation with every operation in dd; theta_w = diag(V_{s-1}) theta
// is formed here from the dd theta (the binary64 thw holds only its hi part).
__device__ __forceinline__ cdd make_reflector_dd(double2* ah, double2* alo, int j, int Nt, int lane) {
  cacc s = cacc0();
  for (int r = j + 1 + lane; r < Nt; r += 64) {
    const cdd x = ldc(ah, alo, r);
    dd::cacc_fmac(s, x, x);
  }
  const ddr s2 = wave_sum_dd(dd::norm(s.re));
  const cdd al = ldc(ah, alo, j);
  if (!(s2.hi > 0.0 || al.im.hi != 0.0)) return czero();
  const ddr nrm = dd::sqrt(dd::add(dd::add(dd::mul(al.re, al.re), dd::mul(al.im, al.im)), s2));
  const ddr be = al.re.hi >= 0.0 ? dd::neg(nrm) : nrm;
  const cdd dz = {dd::sub(al.re, be), al.im};
  const ddr id = dd::div(dd::from(1.0), dd::add(dd::mul(dz.re, dz.re), dd::mul(dz.im, dz.im)));
  const cdd sc = {dd::mul(dz.re, id), dd::neg(dd::mul(dz.im, id))};
  for (int r = j + 1 + lane; r < Nt; r += 64) stc(ah, alo, r, dd::cmul(ldc(ah, alo, r), sc));
  if (lane == 0) stc(ah, alo, j, cdd{be, {0.0, 0.0}});
  return {dd::div(dd::sub(be, al.re), be), dd::div(dd::neg(al.im), be)};
}

constexpr int kCBd = 2;
__device__ __forceinline__ void apply_reflector_cols_dd(double2* Ah, double2* Al, int Nt, int i0, cdd mult, int c0,
                                                        int nc, int lane) {
  const long ov = (long)i0 * Nt;
  const cdd one = {{1.0, 0.0}, {0.0, 0.0}};
  cacc acc[kCBd];
#pragma unroll
  for (int q = 0; q < kCBd; ++q) acc[q] = cacc0();
  for (int r = i0 + lane; r < Nt; r += 64) {
    const cdd vr = r == i0 ? one : ldc(Ah, Al, ov + r);
#pragma unroll
    for (int q = 0; q < kCBd; ++q)
      if (q < nc) dd::cacc_fmac(acc[q], vr, ldc(Ah, Al, (long)(c0 + kQrWaves * q) * Nt + r));
  }
  cdd f[kCBd];
#pragma unroll
  for (int q = 0; q < kCBd; ++q) {
    cdd dot = dd::cnorm(acc[q]);
    dot.re = wave_sum_dd(dot.re);
    dot.im = wave_sum_dd(dot.im);
    f[q] = dd::cmul(mult, dot);
  }
  for (int r = i0 + lane; r < Nt; r += 64) {
    const cdd vr = r == i0 ? one : ldc(Ah, Al, ov + r);
#pragma unroll
    for (int q = 0; q < kCBd; ++q)
      if (q < nc) {
        const long o = (long)(c0 + kQrWaves * q) * Nt + r;
        stc(Ah, Al, o, dd::csub(ldc(Ah, Al, o), dd::cmul(vr, f[q])));
      }
  }
}

__device__ __forceinline__ void finish_q_col_dd(double2* ah, double2* alo, int i, int Nt, cdd ti, int lane) {
  for (int r = lane; r < Nt; r += 64) {
    if (r < i)
      stc(ah, alo, r, czero());
    else if (r == i)
      stc(ah, alo, r, cdd{dd::sub(dd::from(1.0), ti.re), dd::neg(ti.im)});
    else
      stc(ah, alo, r, dd::cmul(cdd{dd::neg(ti.re), dd::neg(ti.im)}, ldc(ah, alo, r)));
  }
}

__global__ __launch_bounds__(kQrThreads) void k_qr_dd(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.x].slot];
  const int M = T.M, Nt = T.Nt;
  double2* __restrict__ Ah = T.Qh;
  double2* __restrict__ Al = T.Qh_lo;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ cdd s_tau[2];

  for (long e = tid; e < (long)M * Nt; e += kQrThreads) {
    const int m = (int)(e % M), n = (int)(e / M);
    const ddr w = {T.lamL[m >> 1], T.lamL_lo[m >> 1]};
    stc(Ah, Al, (long)m * Nt + n, dd::cconj(dd::cscale(ldc(T.thu, T.thu_lo, e), w)));
  }
  __syncthreads();
  if (wave == 0) {
    const cdd t0 = make_reflector_dd(Ah, Al, 0, Nt, lane);
    if (lane == 0) {
      stc(T.tau, T.tau_lo, 0, t0);
      s_tau[0] = t0;
    }
  }
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    const cdd tj = s_tau[j & 1];
    const bool act = tj.re.hi != 0.0 || tj.im.hi != 0.0;
    const cdd ctj = dd::cconj(tj);
    int c0 = j + 1 + wave;
    if (wave == 0 && j + 1 < M) {
      if (act) apply_reflector_cols_dd(Ah, Al, Nt, j, ctj, c0, min(kCBd, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
      __threadfence_block();
      const long on = (long)(j + 1) * Nt;
      const cdd tn = make_reflector_dd(Ah + on, Al + on, j + 1, Nt, lane);
      if (lane == 0) {
        stc(T.tau, T.tau_lo, j + 1, tn);
        s_tau[(j + 1) & 1] = tn;
      }
      c0 += kQrWaves * kCBd;
    }
    if (act)
      for (; c0 < M; c0 += kQrWaves * kCBd)
        apply_reflector_cols_dd(Ah, Al, Nt, j, ctj, c0, min(kCBd, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
    __syncthreads();
  }

  // R^H: dd into Rh (the refinement's W = R^H V), its hi part into thw (FP64 Jacobi)
  for (long e = tid; e < (long)M * M; e += kQrThreads) {
    const int r = (int)(e % M), c = (int)(e / M);
    const cdd v = r >= c ? dd::cconj(ldc(Ah, Al, (long)r * Nt + c)) : czero();
    stc(T.Rh, T.Rh_lo, e, v);
    T.thw[e] = make_double2(v.re.hi, v.im.hi);
  }
  __syncthreads();

  for (int i = M - 1; i >= 0; --i) {
    const cdd ti = ldc(T.tau, T.tau_lo, i);
    const bool act = ti.re.hi != 0.0 || ti.im.hi != 0.0;
    int c0 = i + 1 + wave;
    if (wave == 0 && i + 1 < M) {
      const long on = (long)(i + 1) * Nt;
      finish_q_col_dd(Ah + on, Al + on, i + 1, Nt, ldc(T.tau, T.tau_lo, i + 1), lane);
      __threadfence_block();
      if (act) apply_reflector_cols_dd(Ah, Al, Nt, i, ti, c0, min(kCBd, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
      c0 += kQrWaves * kCBd;
    }
    if (act)
      for (; c0 < M; c0 += kQrWaves * kCBd)
        apply_reflector_cols_dd(Ah, Al, Nt, i, ti, c0, min(kCBd, (M - c0 + kQrWaves - 1) / kQrWaves), lane);
    __syncthreads();
  }
  if (wave == 0) finish_q_col_dd(Ah, Al, 0, Nt, ldc(T.tau, T.tau_lo, 0), lane);
}

struct ZformOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  int k;
  __device__ cdd a(int row, int kk) const { return ldc(t->Qh, t->Qh_lo, (long)kk * t->Nt + row); }
  __device__ cdd b(int kk, int col) const { return ldc(t->V, t->V_lo, (long)t->perm[col] * t->N + kk); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r < t->Nt && c < k) stc(t->Z, t->Z_lo, (long)c * t->Nt + r, v[i][j]);
      }
  }
};

__global__ __launch_bounds__(256) void k_zform_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int k = *t->dim_out;
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->Nt || tn >= k) return;
  ZformOpDD op{t, k};
  ddgemm_tile(op, t->Nt, k, t->N, tm, tn);
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_qr(Task2* d_tasks, const Ent* d_ents, int nent, bool dd, hipStream_t st) {
  if (dd)
    hipLaunchKernelGGL(k_qr_dd, dim3(nent), dim3(kQrThreads), 0, st, d_tasks, d_ents);
  else
    hipLaunchKernelGGL(k_qr, dim3(nent), dim3(kQrThreads), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_zform(Task2* d_tasks, const Ent* d_ents, int nent, int maxNt, int maxK, bool dd, hipStream_t st) {
  if (dd)
    hipLaunchKernelGGL(k_zform_dd, dim3((maxNt + 31) / 32, (maxK + 31) / 32, nent), dim3(256), 0, st, d_tasks,
                       d_ents);
  else
    hipLaunchKernelGGL(k_zform, dim3((maxNt + 63) / 64, (maxK + 63) / 64, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
