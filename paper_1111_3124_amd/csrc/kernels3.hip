// Three-site (U(8)) gate update kernels, FP64 and double-double (gfx950).
//
// The paper treats U(8) gates as elementary (Section 3.1).  On sites s, s+1, s+2:
//   T1 = B_s B_{s+1}                (2a x 2c, kept as (4a x c): rows (alpha, i', j'))
//   theta = (U (x) 1) T1 B_{s+2}    (2a x 4d: rows (alpha, i), columns (j, k, delta))
// Split 1 (s | s+1 s+2) is the two-site machinery on this theta (Jacobi, truncation,
// B_s' = theta Z1_k / nu1, V_s' = sigma / nu1).  The rest, R = Z1_k^H, becomes the
// theta of split 2 (s+1 | s+2): rows (nu, j), columns (k, delta), weighted by the new
// V_s' (k_mid3), and split 2 is an ordinary two-site split.
#include "ddgemm.h"
#include "gemm.h"
#include "kernels3.h"

namespace mpsk {

// ------------------------------------------------------------------ FP64
// T1 = B_s . B_{s+1} with B-operand columns 2*gamma + j'; written as
// T1[(4 alpha + 2 i' + j') + gamma * 4a].
struct T1Op {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ double2 a(int row, int kk) const { return t->Bl[(long)row * t->ldl + kk]; }
  __device__ double2 b(int kk, int col) const { return t->Br[(long)(2 * kk + (col & 1)) * t->ldr + (col >> 1)]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int A4 = 4 * t->a;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + i, al = r >> 1, ip = r & 1;
      if (al >= t->a) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = c0 + j, ga = c >> 1, jp = c & 1;
        if (ga < t->c) t->T1[(long)ga * A4 + (4 * al + 2 * ip + jp)] = acc[i][j];
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_t1(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= 2 * t->a || tn >= 2 * t->c) return;
  T1Op op{t};
  cgemm_tile(op, 2 * t->a, 2 * t->c, t->b, tm, tn);
}

// theta = U-mix of T1 (4a x c) . B_{s+2} (c x 2d), B-operand columns 2*delta + k':
// each thread's 4 x 4 block holds, for one alpha and two deltas, all eight
// (i', j', k') entries.
struct Theta3Op {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ double2 a(int row, int kk) const { return t->T1[(long)kk * 4 * t->a + row]; }
  __device__ double2 b(int kk, int col) const { return t->B3[(long)(2 * kk + (col & 1)) * t->ld3 + (col >> 1)]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int al = r0 >> 2, M = t->M, d = t->d;
    if (al < t->a) {
      const double wl = t->lamL[al];
#pragma unroll
      for (int dd_ = 0; dd_ < 2; ++dd_) {
        const int de = (c0 >> 1) + dd_;
        if (de >= d) continue;
        double2 Tin[8];
#pragma unroll
        for (int ij = 0; ij < 4; ++ij)
#pragma unroll
          for (int kp = 0; kp < 2; ++kp) Tin[ij * 2 + kp] = acc[ij][2 * dd_ + kp];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
          double2 v = cmk(0.0, 0.0);
#pragma unroll
          for (int q = 0; q < 8; ++q) v = cfma(t->U8[o * 8 + q], Tin[q], v);
          const int i = o >> 2, jk = o & 3;
          const long idx = (long)(jk * d + de) * M + (2 * al + i);
          t->thu[idx] = v;
          const double2 w = cscale(v, wl);
          if (t->tr)
            t->thw[(long)(2 * al + i) * t->Nt + (jk * d + de)] = cconj(w);
          else
            t->thw[idx] = w;
        }
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_theta3(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= 4 * t->a || tn >= 2 * t->d) return;
  Theta3Op op{t};
  cgemm_tile(op, 4 * t->a, 2 * t->d, t->c, tm, tn);
}

// theta of split 2 from split 1: theta2[(2 nu + j) + (k d + delta) M2] = conj(Z1[(j,k,delta), nu]),
// (Z1 column nu = the nu-th kept right singular vector of split 1),
// theta2_w = V_s'[nu] theta2.  ents[].slot = split-1 slot, ents[].sweep = split-2 slot.
__global__ __launch_bounds__(256) void k_mid3(Task2* tasks, const Ent* ents) {
  const Task2& A = tasks[ents[blockIdx.z].slot];
  const Task2& Bt = tasks[ents[blockIdx.z].sweep];
  const int k1 = *A.dim_out, d = A.d, N1 = A.Nt, M2 = Bt.M;
  const int nu = blockIdx.y;
  if (nu < k1) {
    const int col = A.perm[nu];
    const double w = A.lamS[nu];
    for (int e = blockIdx.x * 256 + threadIdx.x; e < N1; e += gridDim.x * 256) {
      const int j = e / (2 * d), k = (e / d) & 1, de = e % d;
      const double2 v = cconj(A.Z[(long)col * N1 + e]);
      const long idx = (long)(k * d + de) * M2 + (2 * nu + j);
      Bt.thu[idx] = v;
      const double2 vw = cscale(v, w);
      if (Bt.tr)
        Bt.thw[(long)(2 * nu + j) * Bt.Nt + (k * d + de)] = cconj(vw);
      else
        Bt.thw[idx] = vw;
    }
  }
}

// ------------------------------------------------------------------ double-double
struct T1OpDD {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ cdd a(int row, int kk) const { return ldc(t->Bl, t->Bl_lo, (long)row * t->ldl + kk); }
  __device__ cdd b(int kk, int col) const {
    return ldc(t->Br, t->Br_lo, (long)(2 * kk + (col & 1)) * t->ldr + (col >> 1));
  }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const int A4 = 4 * t->a;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = r0 + i, al = r >> 1, ip = r & 1;
      if (al >= t->a) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = c0 + j, ga = c >> 1, jp = c & 1;
        if (ga < t->c) stc(t->T1, t->T1_lo, (long)ga * A4 + (4 * al + 2 * ip + jp), v[i][j]);
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_t1_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= 2 * t->a || tn >= 2 * t->c) return;
  T1OpDD op{t};
  ddgemm_tile(op, 2 * t->a, 2 * t->c, t->b, tm, tn);
}

// 64 x 32 tiles with 4 x 2 register blocks: one alpha and one delta per thread
struct Theta3OpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ cdd a(int row, int kk) const { return ldc(t->T1, t->T1_lo, (long)kk * 4 * t->a + row); }
  __device__ cdd b(int kk, int col) const {
    return ldc(t->B3, t->B3_lo, (long)(2 * kk + (col & 1)) * t->ld3 + (col >> 1));
  }
  __device__ void epilogue(int r0, int c0, cdd (&T8)[4][2]) const {
    const int al = r0 >> 2, de = c0 >> 1, M = t->M, d = t->d;
    if (al < t->a && de < d) {
      const ddr wl = {t->lamL[al], t->lamL_lo[al]};
      cdd Tin[8];
#pragma unroll
      for (int ij = 0; ij < 4; ++ij)
#pragma unroll
        for (int kp = 0; kp < 2; ++kp) Tin[ij * 2 + kp] = T8[ij][kp];
      for (int o = 0; o < 8; ++o) {
        cacc acc = cacc0();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double2 uh = t->U8[o * 8 + q], ul = t->U8_lo[o * 8 + q];
          dd::cacc_fma(acc, cdd{{uh.x, ul.x}, {uh.y, ul.y}}, Tin[q]);
        }
        const cdd v = dd::cnorm(acc);
        const int i = o >> 2, jk = o & 3;
        const long idx = (long)(jk * d + de) * M + (2 * al + i);
        stc(t->thu, t->thu_lo, idx, v);
        const cdd w = dd::cscale(v, wl);
        if (t->tr)
          t->thw[(long)(2 * al + i) * t->Nt + (jk * d + de)] = make_double2(w.re.hi, -w.im.hi);
        else
          t->thw[idx] = make_double2(w.re.hi, w.im.hi);
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_theta3_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 32;
  if (tm >= 4 * t->a || tn >= 2 * t->d) return;
  Theta3OpDD op{t};
  ddgemm_tile_rb<4, 2>(op, 4 * t->a, 2 * t->d, t->c, tm, tn);
}

__global__ __launch_bounds__(256) void k_mid3_dd(Task2* tasks, const Ent* ents) {
  const Task2& A = tasks[ents[blockIdx.z].slot];
  const Task2& Bt = tasks[ents[blockIdx.z].sweep];
  const int k1 = *A.dim_out, d = A.d, N1 = A.Nt, M2 = Bt.M;
  const int nu = blockIdx.y;
  if (nu < k1) {
    const int col = A.perm[nu];
    const ddr w = {A.lamS[nu], A.lamS_lo[nu]};
    for (int e = blockIdx.x * 256 + threadIdx.x; e < N1; e += gridDim.x * 256) {
      const int j = e / (2 * d), k = (e / d) & 1, de = e % d;
      const cdd v = dd::cconj(ldc(A.Z, A.Z_lo, (long)col * N1 + e));
      const long idx = (long)(k * d + de) * M2 + (2 * nu + j);
      stc(Bt.thu, Bt.thu_lo, idx, v);
      const cdd vw = dd::cscale(v, w);
      if (Bt.tr)
        Bt.thw[(long)(2 * nu + j) * Bt.Nt + (k * d + de)] = make_double2(vw.re.hi, -vw.im.hi);
      else
        Bt.thw[idx] = make_double2(vw.re.hi, vw.im.hi);
    }
  }
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_theta3(Task2* d_tasks, const Ent* d_ents, int nent, int maxA, int maxC, int maxD, bool dd,
                         hipStream_t st) {
  if (dd) {
    hipLaunchKernelGGL(k_t1_dd, dim3((2 * maxA + 31) / 32, (2 * maxC + 31) / 32, nent), dim3(256), 0, st, d_tasks,
                       d_ents);
    MPS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_theta3_dd, dim3((4 * maxA + 63) / 64, (2 * maxD + 31) / 32, nent), dim3(256), 0, st,
                       d_tasks, d_ents);
  } else {
    hipLaunchKernelGGL(k_t1, dim3((2 * maxA + 63) / 64, (2 * maxC + 63) / 64, nent), dim3(256), 0, st, d_tasks,
                       d_ents);
    MPS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_theta3, dim3((4 * maxA + 63) / 64, (2 * maxD + 63) / 64, nent), dim3(256), 0, st,
                       d_tasks, d_ents);
  }
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_mid3(Task2* d_tasks, const Ent* d_ents, int nent, int maxN1, int maxK1, bool dd, hipStream_t st) {
  const dim3 grid((maxN1 + 255) / 256, maxK1, nent);
  if (dd)
    hipLaunchKernelGGL(k_mid3_dd, grid, dim3(256), 0, st, d_tasks, d_ents);
  else
    hipLaunchKernelGGL(k_mid3, grid, dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
