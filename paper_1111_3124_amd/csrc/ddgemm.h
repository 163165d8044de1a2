// Double-double complex GEMM tile and dd load/store helpers shared by the dd kernels.
#pragma once
#include "common.h"
#include "dd.h"

namespace mpsk {

using dd::cacc;
using dd::cdd;
using dd::ddr;

__device__ __forceinline__ cdd ldc(const double2* hi, const double2* lo, long i) {
  const double2 h = hi[i];
  const double2 l = lo ? lo[i] : make_double2(0.0, 0.0);
  return {{h.x, l.x}, {h.y, l.y}};
}
__device__ __forceinline__ void stc(double2* hi, double2* lo, long i, cdd v) {
  hi[i] = make_double2(v.re.hi, v.im.hi);
  lo[i] = make_double2(v.re.lo, v.im.lo);
}
__device__ __forceinline__ cdd czero() { return {{0.0, 0.0}, {0.0, 0.0}}; }
__device__ __forceinline__ cacc cacc0() { return {{0.0, 0.0}, {0.0, 0.0}}; }
__device__ __forceinline__ cdd ld_gate(const double2* U, const double2* Ul, int e) {
  return {{U[e].x, Ul[e].x}, {U[e].y, Ul[e].y}};
}

// ------------------------------------------------------------------ dd GEMM tile
// C (m x n) = A B with dd operands: a (16 RM) x (16 RN) output tile per 256-thread
// block, an RM x RN register block per thread, K slices of 16 staged through LDS as
// hi / lo planes; exact hi*hi products, binary64 cross terms (dd::cacc_fma).
template <int RM, int RN, class Op>
__device__ __forceinline__ void ddgemm_tile_rb(const Op& op, int m, int n, int kd, int tm, int tn) {
  constexpr int TM = 16 * RM, TN = 16 * RN;
  __shared__ double2 Ah[16][TM + 1], Al[16][TM + 1], Bh[16][TN + 1], Bl[16][TN + 1];
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  cacc acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) acc[i][j] = cacc0();
  for (int k0 = 0; k0 < kd; k0 += 16) {
#pragma unroll
    for (int q = 0; q < RM; ++q) {
      const int e = tid + 256 * q;
      int row, kk;
      if (Op::kARowFast) { row = e % TM; kk = e / TM; } else { kk = e & 15; row = e >> 4; }
      const int gr = tm + row, gk = k0 + kk;
      const cdd v = (gr < m && gk < kd) ? op.a(gr, gk) : czero();
      Ah[kk][row] = make_double2(v.re.hi, v.im.hi);
      Al[kk][row] = make_double2(v.re.lo, v.im.lo);
    }
#pragma unroll
    for (int q = 0; q < RN; ++q) {
      const int e = tid + 256 * q;
      int col, kk;
      if (Op::kBColFast) { col = e % TN; kk = e / TN; } else { kk = e & 15; col = e >> 4; }
      const int gc = tn + col, gk = k0 + kk;
      const cdd v = (gc < n && gk < kd) ? op.b(gk, gc) : czero();
      Bh[kk][col] = make_double2(v.re.hi, v.im.hi);
      Bl[kk][col] = make_double2(v.re.lo, v.im.lo);
    }
    __syncthreads();
    for (int kk = 0; kk < 16; ++kk) {
      cdd av[RM], bv[RN];
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const double2 h = Ah[kk][tr * RM + i], l = Al[kk][tr * RM + i];
        av[i] = {{h.x, l.x}, {h.y, l.y}};
      }
#pragma unroll
      for (int j = 0; j < RN; ++j) {
        const double2 h = Bh[kk][tc * RN + j], l = Bl[kk][tc * RN + j];
        bv[j] = {{h.x, l.x}, {h.y, l.y}};
      }
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) dd::cacc_fma(acc[i][j], av[i], bv[j]);
    }
    __syncthreads();
  }
  cdd out[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) out[i][j] = dd::cnorm(acc[i][j]);
  op.epilogue(tm + tr * RM, tn + tc * RN, out);
}

template <class Op>
__device__ __forceinline__ void ddgemm_tile(const Op& op, int m, int n, int kd, int tm, int tn) {
  ddgemm_tile_rb<2, 2>(op, m, n, kd, tm, tn);
}

}  // namespace mpsk
