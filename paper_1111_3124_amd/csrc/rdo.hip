// Reduced density operators (gfx950), FP64 and double-double.
//
// rho = Tr_{other qubits} |Psi><Psi| for a list of qubits (the paper's RDO(list) and
// RDO_block(a, b), Section 3.2), with |Psi> = B_0 B_1 ... B_{n-1} (Eq. (1) in the B
// gauge).  The double layer is contracted without assuming a canonical form:
//   left environment, sites 0 .. q_max:  E[d][beta][beta'], d = (I, I') the open ket
//     and bra indices of the listed sites seen so far (D = 4^l blocks);
//       F[d][i] = E[d]^T B_s[i]                                      (k_rdo_f)
//       listed site:  E'[(I i, I' i')] = F[d][i]^T conj(B_s[i'])     (k_rdo_eo)
//       other site:   E'[d] = sum_i F[d][i]^T conj(B_s[i])          (k_rdo_et)
//   right environment, sites n-1 .. q_max+1:
//       R' = sum_i B_s[i] R B_s[i]^H                                 (k_rdo_g, k_rdo_r)
//   rho[d] = sum_{beta, beta'} E[d][beta][beta'] R[beta][beta']     (k_rdo_fin)
// Every contraction is a batched complex GEMM tile (64 x 64 FP64, 32 x 32 dd).
// Layouts: E[d] and R row-major (m x m); F[d][i] row-major (m_l x m_r); B_s[i][a][b]
// at B[(a * 2 + i) * ld + b].
#include "dd.h"
#include "ddgemm.h"
#include "gemm.h"
#include "rdo.h"

namespace mpsk {

// ------------------------------------------------------------------ FP64
struct RdoFOp {  // F[d][i] (ml x mr) = E[d]^T (ml x ml) B_i (ml x mr)
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d, i;
  __device__ double2 a(int row, int kk) const { return p.E[((long)d * p.ml + kk) * p.ml + row]; }
  __device__ double2 b(int kk, int col) const { return p.B[(long)(kk * 2 + i) * p.ld + col]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    double2* F = p.F + ((long)d * 2 + i) * p.ml * p.mr;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (r0 + r < p.ml && c0 + c < p.mr) F[(long)(r0 + r) * p.mr + c0 + c] = acc[r][c];
  }
};

__global__ __launch_bounds__(256) void k_rdo_f(const RdoStep p) {
  const int z = blockIdx.z, tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= p.ml || tn >= p.mr) return;
  RdoFOp op{p, z >> 1, z & 1};
  cgemm_tile(op, p.ml, p.mr, p.ml, tm, tn);
}

// listed site: E'[d'][b][b'] = sum_a' F[d][i][a'][b] conj(B[a'][i'][b'])
struct RdoEOOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d, i, ip;
  __device__ double2 a(int row, int kk) const {
    return p.F[(((long)d * 2 + i) * p.ml + kk) * p.mr + row];
  }
  __device__ double2 b(int kk, int col) const { return cconj(p.B[(long)(kk * 2 + ip) * p.ld + col]); }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int I = d >> p.l, Ip = d & ((1 << p.l) - 1);
    const long dn = ((long)(2 * I + i) << (p.l + 1)) + (2 * Ip + ip);
    double2* En = p.En + dn * p.mr * p.mr;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (r0 + r < p.mr && c0 + c < p.mr) En[(long)(r0 + r) * p.mr + c0 + c] = acc[r][c];
  }
};

__global__ __launch_bounds__(256) void k_rdo_eo(const RdoStep p) {
  const int z = blockIdx.z, tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= p.mr || tn >= p.mr) return;
  RdoEOOp op{p, z >> 2, (z >> 1) & 1, z & 1};
  cgemm_tile(op, p.mr, p.mr, p.ml, tm, tn);
}

// other site: E'[d][b][b'] = sum_{i, a'} F[d][i][a'][b] conj(B[a'][i][b']), k = (i, a')
struct RdoETOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d;
  __device__ double2 a(int row, int kk) const {
    const int i = kk / p.ml, ap = kk - i * p.ml;
    return p.F[(((long)d * 2 + i) * p.ml + ap) * p.mr + row];
  }
  __device__ double2 b(int kk, int col) const {
    const int i = kk / p.ml, ap = kk - i * p.ml;
    return cconj(p.B[(long)(ap * 2 + i) * p.ld + col]);
  }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    double2* En = p.En + (long)d * p.mr * p.mr;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (r0 + r < p.mr && c0 + c < p.mr) En[(long)(r0 + r) * p.mr + c0 + c] = acc[r][c];
  }
};

__global__ __launch_bounds__(256) void k_rdo_et(const RdoStep p) {
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= p.mr || tn >= p.mr) return;
  RdoETOp op{p, (int)blockIdx.z};
  cgemm_tile(op, p.mr, p.mr, 2 * p.ml, tm, tn);
}

// right environment: G_i = B_i R (ml x mr), then R' = sum_i G_i B_i^H (ml x ml)
struct RdoGOp {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int i;
  __device__ double2 a(int row, int kk) const { return p.B[(long)(row * 2 + i) * p.ld + kk]; }
  __device__ double2 b(int kk, int col) const { return p.E[(long)kk * p.mr + col]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    double2* G = p.F + (long)i * p.ml * p.mr;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (r0 + r < p.ml && c0 + c < p.mr) G[(long)(r0 + r) * p.mr + c0 + c] = acc[r][c];
  }
};

__global__ __launch_bounds__(256) void k_rdo_g(const RdoStep p) {
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= p.ml || tn >= p.mr) return;
  RdoGOp op{p, (int)blockIdx.z};
  cgemm_tile(op, p.ml, p.mr, p.mr, tm, tn);
}

struct RdoROp {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = false;
  RdoStep p;
  __device__ double2 a(int row, int kk) const {
    const int i = kk / p.mr, b = kk - i * p.mr;
    return p.F[((long)i * p.ml + row) * p.mr + b];
  }
  __device__ double2 b(int kk, int col) const {
    const int i = kk / p.mr, b = kk - i * p.mr;
    return cconj(p.B[(long)(col * 2 + i) * p.ld + b]);
  }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (r0 + r < p.ml && c0 + c < p.ml) p.En[(long)(r0 + r) * p.ml + c0 + c] = acc[r][c];
  }
};

__global__ __launch_bounds__(256) void k_rdo_r(const RdoStep p) {
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= p.ml || tn >= p.ml) return;
  RdoROp op{p};
  cgemm_tile(op, p.ml, p.ml, 2 * p.mr, tm, tn);
}

// rho[d] = sum_{b, b'} E[d][b][b'] R[b][b']: a block per d (fixed reduction order)
__global__ __launch_bounds__(256) void k_rdo_fin(const RdoStep p) {
  const int d = blockIdx.x, m = p.mr, tid = threadIdx.x;
  const double2* Ed = p.E + (long)d * m * m;
  double2 s = cmk(0.0, 0.0);
  for (long e = tid; e < (long)m * m; e += 256) s = cfma(Ed[e], p.F[e], s);
  __shared__ double2 red[256];
  red[tid] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) red[tid] = cadd(red[tid], red[tid + k]);
    __syncthreads();
  }
  if (tid == 0) p.En[d] = red[0];
}

// ------------------------------------------------------------------ double-double
struct RdoFOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d, i;
  __device__ cdd a(int row, int kk) const { return ldc(p.E, p.Elo, ((long)d * p.ml + kk) * p.ml + row); }
  __device__ cdd b(int kk, int col) const { return ldc(p.B, p.Blo, (long)(kk * 2 + i) * p.ld + col); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const long o = ((long)d * 2 + i) * p.ml * p.mr;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (r0 + r < p.ml && c0 + c < p.mr) stc(p.F, p.Flo, o + (long)(r0 + r) * p.mr + c0 + c, v[r][c]);
  }
};

__global__ __launch_bounds__(256) void k_rdo_f_dd(const RdoStep p) {
  const int z = blockIdx.z, tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= p.ml || tn >= p.mr) return;
  RdoFOpDD op{p, z >> 1, z & 1};
  ddgemm_tile(op, p.ml, p.mr, p.ml, tm, tn);
}

struct RdoEOOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d, i, ip;
  __device__ cdd a(int row, int kk) const {
    return ldc(p.F, p.Flo, (((long)d * 2 + i) * p.ml + kk) * p.mr + row);
  }
  __device__ cdd b(int kk, int col) const {
    return dd::cconj(ldc(p.B, p.Blo, (long)(kk * 2 + ip) * p.ld + col));
  }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const int I = d >> p.l, Ip = d & ((1 << p.l) - 1);
    const long dn = ((long)(2 * I + i) << (p.l + 1)) + (2 * Ip + ip);
    const long o = dn * p.mr * p.mr;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (r0 + r < p.mr && c0 + c < p.mr) stc(p.En, p.Enlo, o + (long)(r0 + r) * p.mr + c0 + c, v[r][c]);
  }
};

__global__ __launch_bounds__(256) void k_rdo_eo_dd(const RdoStep p) {
  const int z = blockIdx.z, tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= p.mr || tn >= p.mr) return;
  RdoEOOpDD op{p, z >> 2, (z >> 1) & 1, z & 1};
  ddgemm_tile(op, p.mr, p.mr, p.ml, tm, tn);
}

struct RdoETOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int d;
  __device__ cdd a(int row, int kk) const {
    const int i = kk / p.ml, ap = kk - i * p.ml;
    return ldc(p.F, p.Flo, (((long)d * 2 + i) * p.ml + ap) * p.mr + row);
  }
  __device__ cdd b(int kk, int col) const {
    const int i = kk / p.ml, ap = kk - i * p.ml;
    return dd::cconj(ldc(p.B, p.Blo, (long)(ap * 2 + i) * p.ld + col));
  }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const long o = (long)d * p.mr * p.mr;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (r0 + r < p.mr && c0 + c < p.mr) stc(p.En, p.Enlo, o + (long)(r0 + r) * p.mr + c0 + c, v[r][c]);
  }
};

__global__ __launch_bounds__(256) void k_rdo_et_dd(const RdoStep p) {
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= p.mr || tn >= p.mr) return;
  RdoETOpDD op{p, (int)blockIdx.z};
  ddgemm_tile(op, p.mr, p.mr, 2 * p.ml, tm, tn);
}

struct RdoGOpDD {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  RdoStep p;
  int i;
  __device__ cdd a(int row, int kk) const { return ldc(p.B, p.Blo, (long)(row * 2 + i) * p.ld + kk); }
  __device__ cdd b(int kk, int col) const { return ldc(p.E, p.Elo, (long)kk * p.mr + col); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const long o = (long)i * p.ml * p.mr;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (r0 + r < p.ml && c0 + c < p.mr) stc(p.F, p.Flo, o + (long)(r0 + r) * p.mr + c0 + c, v[r][c]);
  }
};

__global__ __launch_bounds__(256) void k_rdo_g_dd(const RdoStep p) {
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= p.ml || tn >= p.mr) return;
  RdoGOpDD op{p, (int)blockIdx.z};
  ddgemm_tile(op, p.ml, p.mr, p.mr, tm, tn);
}

struct RdoROpDD {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = false;
  RdoStep p;
  __device__ cdd a(int row, int kk) const {
    const int i = kk / p.mr, b = kk - i * p.mr;
    return ldc(p.F, p.Flo, ((long)i * p.ml + row) * p.mr + b);
  }
  __device__ cdd b(int kk, int col) const {
    const int i = kk / p.mr, b = kk - i * p.mr;
    return dd::cconj(ldc(p.B, p.Blo, (long)(col * 2 + i) * p.ld + b));
  }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (r0 + r < p.ml && c0 + c < p.ml) stc(p.En, p.Enlo, (long)(r0 + r) * p.ml + c0 + c, v[r][c]);
  }
};

__global__ __launch_bounds__(256) void k_rdo_r_dd(const RdoStep p) {
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= p.ml || tn >= p.ml) return;
  RdoROpDD op{p};
  ddgemm_tile(op, p.ml, p.ml, 2 * p.mr, tm, tn);
}

__global__ __launch_bounds__(256) void k_rdo_fin_dd(const RdoStep p) {
  const int d = blockIdx.x, m = p.mr, tid = threadIdx.x;
  const long o = (long)d * m * m;
  cacc s = cacc0();
  for (long e = tid; e < (long)m * m; e += 256) dd::cacc_fma(s, ldc(p.E, p.Elo, o + e), ldc(p.F, p.Flo, e));
  __shared__ ddr rr[256], ri[256];
  rr[tid] = dd::norm(s.re);
  ri[tid] = dd::norm(s.im);
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (tid < k) {
      rr[tid] = dd::add(rr[tid], rr[tid + k]);
      ri[tid] = dd::add(ri[tid], ri[tid + k]);
    }
    __syncthreads();
  }
  if (tid == 0) stc(p.En, p.Enlo, d, cdd{rr[0], ri[0]});
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

static int tiles(int n, int t) { return (n + t - 1) / t; }

hipError_t launch_rdo_left(const RdoStep& p, int D, bool open, bool dd, hipStream_t st) {
  const int t = dd ? 32 : 64;
  if (dd)
    hipLaunchKernelGGL(k_rdo_f_dd, dim3(tiles(p.ml, t), tiles(p.mr, t), 2 * D), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(k_rdo_f, dim3(tiles(p.ml, t), tiles(p.mr, t), 2 * D), dim3(256), 0, st, p);
  MPS_LAUNCH_CHECK();
  if (open) {
    if (dd)
      hipLaunchKernelGGL(k_rdo_eo_dd, dim3(tiles(p.mr, t), tiles(p.mr, t), 4 * D), dim3(256), 0, st, p);
    else
      hipLaunchKernelGGL(k_rdo_eo, dim3(tiles(p.mr, t), tiles(p.mr, t), 4 * D), dim3(256), 0, st, p);
  } else {
    if (dd)
      hipLaunchKernelGGL(k_rdo_et_dd, dim3(tiles(p.mr, t), tiles(p.mr, t), D), dim3(256), 0, st, p);
    else
      hipLaunchKernelGGL(k_rdo_et, dim3(tiles(p.mr, t), tiles(p.mr, t), D), dim3(256), 0, st, p);
  }
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_rdo_right(const RdoStep& p, bool dd, hipStream_t st) {
  const int t = dd ? 32 : 64;
  if (dd)
    hipLaunchKernelGGL(k_rdo_g_dd, dim3(tiles(p.ml, t), tiles(p.mr, t), 2), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(k_rdo_g, dim3(tiles(p.ml, t), tiles(p.mr, t), 2), dim3(256), 0, st, p);
  MPS_LAUNCH_CHECK();
  if (dd)
    hipLaunchKernelGGL(k_rdo_r_dd, dim3(tiles(p.ml, t), tiles(p.ml, t), 1), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(k_rdo_r, dim3(tiles(p.ml, t), tiles(p.ml, t), 1), dim3(256), 0, st, p);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_rdo_final(const RdoStep& p, int D, bool dd, hipStream_t st) {
  if (dd)
    hipLaunchKernelGGL(k_rdo_fin_dd, dim3(D), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(k_rdo_fin, dim3(D), dim3(256), 0, st, p);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
