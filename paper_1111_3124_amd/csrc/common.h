// Shared device/host definitions of the gate-update kernels (gfx950).
//
// Layouts (device memory):
//   site tensor B_s[alpha][i][beta]  at  B[(alpha*2 + i)*ld + beta], complex double2,
//                                     ld = capacity of the site's right bond;
//   theta (M x Nt), column-major, ld = M (compact to the live dims);
//     2-site rows r = 2*alpha + i (M = 2a), columns col = j*c + gamma (Nt = 2c);
//   the Jacobi problem W (JM x N) with V (N x N), column-major: W = theta_w (JM = M,
//     N = Nt), or for a wide theta (Nt > M) W = theta_w^H (JM = Nt, N = M);
//   Z (Nt x N), column-major, ld = Nt: the right singular vectors the split uses.
// A double-double handle keeps a second "lo" plane beside every hi array.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpsk {

constexpr int kMaxSort = 4096;  // largest N the truncation kernel sorts in LDS

// ------------------------------------------------------------------ complex FP64
__host__ __device__ inline double2 cmk(double x, double y) { return make_double2(x, y); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__host__ __device__ inline double2 cfma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__host__ __device__ inline double2 cfmac(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}

// ------------------------------------------------------------------ task descriptors
// One two-site update (one SVD) of a wave.  The host fills these and copies the
// array to the device; kernels index it with blockIdx.y / blockIdx.z.
struct Task2 {
  // state
  double2* Bl;          // site s
  double2* Br;          // site s+1
  double2* Bl_lo;       // dd lo planes (null on FP64 handles)
  double2* Br_lo;
  int ldl, ldr;         // row lengths of Bl, Br
  int a, b, c;          // live bond dims m_{s-1}, m_s, m_{s+1}
  int M, Nt;            // theta rows (2a) and columns (2c, or 4d: three-site first split)
  int JM, N;            // Jacobi problem rows and columns: (M, Nt), or (Nt, M) when tr
  int tr;               // 1: wide theta, the Jacobi runs on theta_w^H
  const double* lamL;   // V_{s-1}: a values (boundary: a 1)
  const double* lamL_lo;
  double* lamS;         // V_s output slot
  double* lamS_lo;
  int* dim_out;         // where the new m_s goes (device bond-dim table)
  int chi;              // truncation: chi_max and eps of the state this task updates
  double eps;
  // gate, row-major 4x4
  double2 U[16];
  double2 U_lo[16];
  // workspace (compact, sized for this task)
  double2* thu;         // theta unweighted, M x N
  double2* thw;         // theta weighted by V_{s-1}; becomes W = thw V
  double2* V;           // N x N
  double2* thu_lo;      // dd planes of the above (dd handles)
  double2* thw_lo;
  double2* V_lo;
  // right factor of the split (Nt rows; column perm[nu] is the nu-th kept one): V, or
  // for a wide theta W itself, whose kept columns are scaled to unit norm
  double2* Z;
  double2* Z_lo;
  double2* aux1;        // dd handles: N x N scratch (V^H V - I), binary64
  double2* aux3;        // dd handles: M x N scratch (refinement products), binary64
  double2* aux2;        // dd handles: N x N scratch (V (V^H V - I)), binary64
  double* sig2;         // N: squared column norms of W (from the Jacobi Gram diagonals)
  double* sig2_lo;
  int* perm;            // N: column order, sigma descending
  double* fro2;         // ||thw||_F^2 (zero-column threshold)
  double* frop;         // its partial sums, one per chunk of kFroChunk elements of thw
  double* stats;        // 8 doubles: W, w, gap, epsdist, k, rank, nu (hi, lo)
  int* flags;           // 3 ints: rotation flags of the current / next / previous sweep
  // three-site gates (first split): theta is 2a x 4d, columns (j*2 + k)*d + delta
  const double2* B3;    // site s+2 (null for a two-site update)
  const double2* B3_lo;
  int ld3, d;           // row length of B3, m_{s+2}
  const double2* U8;    // 8 x 8 gate, row-major (device copy)
  const double2* U8_lo;
  double2* T1;          // scratch: B_s B_{s+1} as (4a x c), column-major
  double2* T1_lo;
  // the Jacobi step's operands: W (JR x N, column-major) and, when jvec, V (N x N);
  // W = thw, V = V, JR = JM unless the problem is preconditioned by QR
  double2* JW;
  double2* JV;
  int JR, jvec;
  // the split Jacobi step's partial Grams: per column-block pair and row half, the
  // 16 x 16 Re part and P = Xr^T Xi part (2 x 2 x 256 doubles a pair)
  double* JG;
  // V's rotations deferred by one step (fused step, block width 8): per step parity and
  // column-block pair, R (16 x 16, row-major) in VPR and in VPC the pair's 16 columns
  // and a tag (one more than the global step g = sweep * steps + step that wrote it;
  // 0 once applied or when nothing rotated)
  double2* VPR;
  int* VPC;
  // QR preconditioning (qr = 1): column order, reflector heads, scales, panel factors
  int qr;
  int* qperm;
  double2* qvd;
  double* qt;
  double2* qT;
};

// ||theta_w||_F^2 is summed over fixed chunks of thw (partials in a per-task array,
// then added in chunk order), so that it does not depend on how a launch is shaped
constexpr int kFroChunk = 4096;

// One entry of a launch list: the task slot a block row works on and, for the
// Jacobi steps, the slot's current sweep index.
struct Ent {
  int slot;
  int sweep;
};

// One single-site gate.
struct Task1 {
  double2* B;
  double2* B_lo;
  int ld, a, b;
  double2 U[4];
  double2 U_lo[4];
};

}  // namespace mpsk
