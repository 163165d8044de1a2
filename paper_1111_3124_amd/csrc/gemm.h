// Complex FP64 GEMM tile shared by the gate-update kernels.
#pragma once
#include "common.h"

namespace mpsk {

// ------------------------------------------------------------------ complex GEMM tile
// C (m x n) = A (m x kd) B (kd x n), one 64 x 64 output tile per 256-thread block,
// each thread a 4 x 4 register block (rows tr*4.., columns tc*4..).  Operands are
// staged through LDS in K slices of 16.  Op supplies the element loaders, which
// index varies fastest across threads in each load (for coalescing), and the
// epilogue that consumes the 4 x 4 block.
template <class Op>
__device__ __forceinline__ void cgemm_tile(const Op& op, int m, int n, int kd, int tm, int tn) {
  __shared__ double2 As[16][64 + 1];
  __shared__ double2 Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = cmk(0.0, 0.0);
  for (int k0 = 0; k0 < kd; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int row, kk;
      if (Op::kARowFast) { row = e & 63; kk = e >> 6; } else { kk = e & 15; row = e >> 4; }
      const int gr = tm + row, gk = k0 + kk;
      As[kk][row] = (gr < m && gk < kd) ? op.a(gr, gk) : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int col, kk;
      if (Op::kBColFast) { col = e & 63; kk = e >> 6; } else { kk = e & 15; col = e >> 4; }
      const int gc = tn + col, gk = k0 + kk;
      Bs[kk][col] = (gc < n && gk < kd) ? op.b(gk, gc) : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cfma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  op.epilogue(tm + tr * 4, tn + tc * 4, acc);
}

}  // namespace mpsk
