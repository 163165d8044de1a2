// HIP kernels (gfx950) of the two-site and single-site gate update, FP64.
//
// The update follows the paper's Section 3.1 (a U(4) gate on qubits s, s+1 changes
// only Q_s, V_s, Q_{s+1}; small Schmidt coefficients are truncated), in the
// division-free right-canonical gauge B_s = Q_s V_s:
//   theta  = (U (x) 1) B_s B_{s+1}                     [k_theta2: GEMM + U epilogue]
//   theta_w = diag(V_{s-1}) theta
//   theta_w V = W with orthogonal columns              [k_jacobi_step: block one-sided Jacobi]
//   sigma_j = ||W_j|| sorted, truncated, renormalised  [k_truncate]
//   B_{s+1}' = Z_k^H,  B_s' = theta Z_k / nu,  V_s' = sigma_k / nu   [k_split_*]
// Z = V (columns permuted by sigma).  Since theta_w Z_k = X_k Sigma_k, B_s' equals
// the paper's Q_s' V_s' without ever dividing by a Schmidt value.
#include "common.h"
#include "launch.h"

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

// ------------------------------------------------------------------ prep
// V = I_N, zero the Frobenius accumulator and the rotation flags.
__global__ __launch_bounds__(256) void k_prep2(Task2* tasks) {
  const Task2& T = tasks[blockIdx.y];
  const int N = T.N;
  const long nn = (long)N * N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
    const int r = (int)(e % N), c = (int)(e / N);
    T.V[e] = cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *T.fro2 = 0.0;
    T.flags[0] = T.flags[1] = T.flags[2] = 0;
  }
}

// ------------------------------------------------------------------ theta (2 sites)
// T = B_s (2a x b) . B_{s+1} (b x 2c) with the B-operand columns ordered 2*gamma + j',
// so each thread's 4 x 4 block holds, for two alphas and two gammas, all four
// (i', j') entries; the epilogue mixes them with U and writes theta and theta_w.
struct ThetaOp {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ double2 a(int row, int kk) const { return t->Bl[(long)row * t->ldl + kk]; }
  __device__ double2 b(int kk, int col) const {
    return t->Br[(long)(2 * kk + (col & 1)) * t->ldr + (col >> 1)];
  }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int a_ = t->a, c_ = t->c, M = t->M;
    double fro = 0.0;
#pragma unroll
    for (int da = 0; da < 2; ++da) {
      const int al = (r0 >> 1) + da;
      if (al >= a_) continue;
      const double wl = t->lamL[al];
#pragma unroll
      for (int dg = 0; dg < 2; ++dg) {
        const int ga = (c0 >> 1) + dg;
        if (ga >= c_) continue;
        double2 Tin[4];
#pragma unroll
        for (int ip = 0; ip < 2; ++ip)
#pragma unroll
          for (int jp = 0; jp < 2; ++jp) Tin[ip * 2 + jp] = acc[2 * da + ip][2 * dg + jp];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            double2 o = cmk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 4; ++q) o = cfma(t->U[(i * 2 + j) * 4 + q], Tin[q], o);
            const long idx = (long)(j * c_ + ga) * M + (2 * al + i);
            t->thu[idx] = o;
            const double2 ow = cscale(o, wl);
            t->thw[idx] = ow;
            fro += ow.x * ow.x + ow.y * ow.y;
          }
      }
    }
    // block reduction of ||theta_w||^2 (zero-column threshold of the Jacobi)
    __shared__ double red[256];
    red[threadIdx.x] = fro;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(t->fro2, red[0]);
  }
};

__global__ __launch_bounds__(256) void k_theta2(Task2* tasks) {
  const Task2* t = &tasks[blockIdx.z];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->M || tn >= t->N) return;
  ThetaOp op{t};
  cgemm_tile(op, t->M, t->N, t->b, tm, tn);
}

// ------------------------------------------------------------------ Jacobi step
// One step of the block one-sided Jacobi sweep.  Columns are grouped in blocks of
// BW; the blocks are paired by the round-robin ("circle") schedule, so that the
// 2*BW-column groups of one step are disjoint and all block pairs meet once per
// sweep.  Each 256-thread block takes one pair of one task:
//   1. G = A_P^H A_P (2BW x 2BW) from the pair's columns A_P of W (LDS row chunks);
//   2. cyclic two-sided Jacobi on G in LDS, R accumulating the rotations
//      (each rotation the complex symmetric Schur 2x2 of Golub & Van Loan 8.4/8.5,
//      applied to columns then rows for the disjoint pairs of a round);
//   3. A_P <- A_P R and V_P <- V_P R (row per thread), and sig2 <- diag(R^H G R).
// A pair whose off-diagonal entries are all below tol * sqrt(G_pp G_qq) is left
// alone; a task whose previous sweep rotated nothing is converged and skipped.
template <int BW>
__global__ __launch_bounds__(256) void k_jacobi_step(Task2* tasks, int step, int sweep, double tol_mult,
                                                      int maxin) {
  constexpr int W2 = 2 * BW;
  static_assert(W2 * W2 == 256, "one Gram entry per thread");
  const Task2& T = tasks[blockIdx.y];
  const int N = T.N, M = T.M;
  const int nb = (N + BW - 1) / BW;
  const int nbp = nb + (nb & 1);
  const int pi = blockIdx.x;
  if (step >= nbp - 1 || pi >= nbp / 2) return;
  int* flags = T.flags;
  const int tid = threadIdx.x;
  // slot (sweep+1)%3 is neither read nor written during this sweep: clear it for the
  // next one (also for converged tasks, whose later sweeps must read 0)
  if (step == 0 && pi == 0 && tid == 0) flags[(sweep + 1) % 3] = 0;
  if (sweep > 0 && flags[(sweep + 2) % 3] == 0) return;

  __shared__ int cols[W2];
  __shared__ double2 Ch[64][W2 + 1];
  __shared__ double2 G[W2][W2 + 1];
  __shared__ double2 R[W2][W2 + 1];
  __shared__ double rc[W2 / 2], rs[W2 / 2];
  __shared__ double2 rev[W2 / 2];
  __shared__ int rp[W2 / 2], rq[W2 / 2], rf[W2 / 2];
  __shared__ int any_rot, sweep_rot;

  auto player = [&](int i, int r, int np) { return i == 0 ? 0 : 1 + (i - 1 + r) % (np - 1); };
  const int I = player(pi, step, nbp), J = player(nbp - 1 - pi, step, nbp);
  if (tid < W2) {
    const int blk = tid < BW ? I : J;
    const int c = blk * BW + (tid % BW);
    cols[tid] = (blk < nb && c < N) ? c : -1;
  }
  if (tid == 0) any_rot = 0;
  __syncthreads();

  const double2* __restrict__ A = T.thw;
  // 1. Gram of the pair
  const int p = tid / W2, q = tid % W2;
  double2 acc = cmk(0.0, 0.0);
  for (int r0 = 0; r0 < M; r0 += 64) {
    for (int e = tid; e < 64 * W2; e += 256) {
      const int rr = e & 63, l = e >> 6;
      const int c = cols[l], r = r0 + rr;
      Ch[rr][l] = (c >= 0 && r < M) ? A[(long)c * M + r] : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 64; ++rr) acc = cfmac(Ch[rr][p], Ch[rr][q], acc);
    __syncthreads();
  }
  G[p][q] = acc;
  R[p][q] = cmk(p == q ? 1.0 : 0.0, 0.0);
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-53;
  const double ztol = *T.fro2 * 0x1p-96;
  __syncthreads();

  // 2. two-sided Jacobi on G (W2 x W2 Hermitian)
  for (int isw = 0; isw < maxin; ++isw) {
    if (tid == 0) sweep_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < W2 - 1; ++rnd) {
      if (tid < W2 / 2) {
        const int pa = player(tid, rnd, W2), pb = player(W2 - 1 - tid, rnd, W2);
        const int pp = pa < pb ? pa : pb, qq = pa < pb ? pb : pa;
        const double al = G[pp][pp].x, be = G[qq][qq].x;
        const double2 g = G[pp][qq];
        const double gabs = hypot(g.x, g.y);
        int rot = cols[pp] >= 0 && cols[qq] >= 0 && al > ztol && be > ztol && gabs > tol * sqrt(al * be);
        rp[tid] = pp; rq[tid] = qq; rf[tid] = rot;
        if (rot) {
          const double zeta = (be - al) / (2.0 * gabs);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          rc[tid] = c;
          rs[tid] = t * c;
          rev[tid] = cmk(g.x / gabs, -g.y / gabs);  // e^{-i phi}
          sweep_rot = 1;
        }
      }
      __syncthreads();
      {  // columns p, q of G (threads 0..127) and of R (threads 128..255)
        const int pr = (tid >> 4) & 7, row = tid & 15;
        if (pr < W2 / 2 && rf[pr]) {
          double2(*X)[W2 + 1] = (tid >> 7) ? R : G;
          const int pp = rp[pr], qq = rq[pr];
          const double c = rc[pr], s = rs[pr];
          const double2 x = X[row][pp], y = X[row][qq];
          const double2 ey = cmul(rev[pr], y);
          X[row][pp] = csub(cscale(x, c), cscale(ey, s));
          X[row][qq] = cadd(cscale(x, s), cscale(ey, c));
        }
      }
      __syncthreads();
      if (tid < 128) {  // rows p, q of G:  G <- J^H G
        const int pr = tid >> 4, col = tid & 15;
        if (pr < W2 / 2 && rf[pr]) {
          const int pp = rp[pr], qq = rq[pr];
          const double c = rc[pr], s = rs[pr];
          const double2 x = G[pp][col], y = G[qq][col];
          const double2 ey = cmul(cconj(rev[pr]), y);
          double2 np_ = csub(cscale(x, c), cscale(ey, s));
          double2 nq_ = cadd(cscale(x, s), cscale(ey, c));
          if (col == qq) np_ = cmk(0.0, 0.0);
          if (col == pp) { nq_ = cmk(0.0, 0.0); np_.y = 0.0; }
          if (col == qq) nq_.y = 0.0;
          G[pp][col] = np_;
          G[qq][col] = nq_;
        }
      }
      __syncthreads();
    }
    if (!sweep_rot) break;
    if (tid == 0) any_rot = 1;
  }
  __syncthreads();

  // 3. apply R to the pair's columns of W and V
  if (any_rot) {
    double2* __restrict__ Aw = T.thw;
    double2* __restrict__ Vw = T.V;
    for (int pass = 0; pass < 2; ++pass) {
      double2* X = pass ? Vw : Aw;
      const int rows = pass ? N : M;
      for (int r = tid; r < rows; r += 256) {
        double2 x[W2];
#pragma unroll
        for (int l = 0; l < W2; ++l) x[l] = cols[l] >= 0 ? X[(long)cols[l] * rows + r] : cmk(0.0, 0.0);
#pragma unroll
        for (int pc = 0; pc < W2; ++pc) {
          double2 y = cmk(0.0, 0.0);
#pragma unroll
          for (int l = 0; l < W2; ++l) y = cfma(x[l], R[l][pc], y);
          if (cols[pc] >= 0) X[(long)cols[pc] * rows + r] = y;
        }
      }
    }
    if (tid == 0) flags[sweep % 3] = 1;
  }
  if (tid < W2 && cols[tid] >= 0) T.sig2[cols[tid]] = G[tid][tid].x;
}

// ------------------------------------------------------------------ truncation
// Sort sigma^2 descending (bitonic, ties by column index), suffix sums for the
// discarded weight, the kept count k = min(chi, k_eps, rank, min(M, N)), the new
// Schmidt values sigma_j / nu and the column order for the split.
__global__ __launch_bounds__(1024) void k_truncate(Task2* tasks, int chi, double eps, double floor_rel) {
  Task2& T = tasks[blockIdx.x];
  const int N = T.N, M = T.M;
  int P = 1;
  while (P < N) P <<= 1;
  __shared__ double key[kMaxSort];
  __shared__ int idx[kMaxSort];
  __shared__ double sc[kMaxSort];
  __shared__ int s_rank, s_keps;
  __shared__ double s_kept;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < P; j += nt) {
    key[j] = j < N ? fmax(T.sig2[j], 0.0) : -1.0;
    idx[j] = j;
  }
  if (tid == 0) { s_rank = 0; s_keps = N; s_kept = 0.0; }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += nt) {
        const int l = i ^ stride;
        if (l > i) {
          const bool before = key[i] > key[l] || (key[i] == key[l] && idx[i] < idx[l]);
          const bool dir = (i & size) == 0;
          if (dir != before) {
            const double tk = key[i]; key[i] = key[l]; key[l] = tk;
            const int ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  // suffix sums: sc[j] = sum_{i >= j} sigma_i^2
  for (int j = tid; j < P; j += nt) sc[j] = j < N ? key[j] : 0.0;
  __syncthreads();
  for (int off = 1; off < P; off <<= 1) {
    double v[kMaxSort / 256];
    int cnt = 0;
    for (int j = tid; j < P; j += nt) v[cnt++] = (j + off < P) ? sc[j + off] : 0.0;
    __syncthreads();
    cnt = 0;
    for (int j = tid; j < P; j += nt) sc[j] += v[cnt++];
    __syncthreads();
  }
  const double W = sc[0];
  const double s0 = sqrt(key[0]);
  const double epsW = eps * W;
  int myrank = 0;
  for (int j = tid; j < N; j += nt) {
    if (sqrt(key[j]) > floor_rel * s0) ++myrank;
    const int kk = j + 1;  // candidate kept count
    const double tailk = kk < N ? sc[kk] : 0.0;
    if (tailk <= epsW) atomicMin(&s_keps, kk);
  }
  atomicAdd(&s_rank, myrank);
  __syncthreads();
  int k = chi;
  if (s_keps < k) k = s_keps;
  if (s_rank < k) k = s_rank;
  const int mn = M < N ? M : N;
  if (mn < k) k = mn;
  if (k < 1) k = 1;
  double part = 0.0;
  for (int j = tid; j < k; j += nt) part += key[j];
  atomicAdd(&s_kept, part);
  __syncthreads();
  const double nu = sqrt(s_kept);
  for (int j = tid; j < N; j += nt) {
    T.perm[j] = idx[j];
    if (j < k) T.lamS[j] = sqrt(key[j]) / nu;
  }
  if (tid == 0) {
    const double tail = k < N ? sc[k] : 0.0;
    double* st = T.stats;
    st[0] = W;
    st[1] = W > 0 ? tail / W : 0.0;
    st[2] = (k < s_rank) ? (sqrt(key[k - 1]) - sqrt(key[k])) / s0 : INFINITY;
    double ed = INFINITY;
    if (eps > 0) {
      for (int kk = s_keps - 1; kk <= s_keps; ++kk) {
        if (kk < 1 || kk > N) continue;
        const double tk = kk < N ? sc[kk] : 0.0;
        const double d = fabs(tk - epsW) / epsW;
        ed = d < ed ? d : ed;
      }
    }
    st[3] = ed;
    st[4] = k;
    st[5] = s_rank;
    st[6] = nu;
    st[7] = 0.0;
    *T.dim_out = k;
  }
}

// ------------------------------------------------------------------ split
// B_{s+1}'[nu][j][gamma] = conj(V[(j c + gamma), perm[nu]])  (rows of Z_k^H)
__global__ __launch_bounds__(256) void k_split_right(Task2* tasks) {
  const Task2& T = tasks[blockIdx.z];
  const int k = *T.dim_out, N = T.N, c = T.c;
  const int nu = blockIdx.y;
  if (nu >= k) return;
  const int col = T.perm[nu];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < N; e += gridDim.x * 256) {
    const int j = e / c, ga = e - j * c;
    T.Br[(long)(2 * nu + j) * T.ldr + ga] = cconj(T.V[(long)col * N + e]);
  }
}

// B_s' = theta Z_k / nu  (M x k), written as B_s'[alpha][i][nu] = row 2 alpha + i.
struct SplitLeftOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  int k;
  double inv_nu;
  __device__ double2 a(int row, int kk) const { return t->thu[(long)kk * t->M + row]; }
  __device__ double2 b(int kk, int col) const { return t->V[(long)t->perm[col] * t->N + kk]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + i;
      if (r >= t->M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cc = c0 + j;
        if (cc < k) t->Bl[(long)r * t->ldl + cc] = cscale(acc[i][j], inv_nu);
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_split_left(Task2* tasks) {
  const Task2* t = &tasks[blockIdx.z];
  const int k = *t->dim_out;
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->M || tn >= k) return;
  SplitLeftOp op{t, k, 1.0 / t->stats[6]};
  cgemm_tile(op, t->M, k, t->N, tm, tn);
}

// ------------------------------------------------------------------ single-site gate
__global__ __launch_bounds__(256) void k_gate1(Task1* tasks) {
  const Task1& T = tasks[blockIdx.y];
  const long nel = (long)T.a * T.b;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nel; e += (long)gridDim.x * 256) {
    const int al = (int)(e / T.b), be = (int)(e - (long)al * T.b);
    double2* p0 = T.B + (long)(2 * al) * T.ld + be;
    double2* p1 = p0 + T.ld;
    const double2 x0 = *p0, x1 = *p1;
    *p0 = cfma(T.U[1], x1, cmul(T.U[0], x0));
    *p1 = cfma(T.U[3], x1, cmul(T.U[2], x0));
  }
}

// ------------------------------------------------------------------ amplitudes
// c(b) = B_0[b_0] B_1[b_1] ... B_{n-1}[b_{n-1}]  (Eq. (1) in the B gauge): one block
// per bitstring, the running row vector in LDS.
__global__ __launch_bounds__(256) void k_amplitude(const AmpArgs args) {
  __shared__ double2 v[1024], w[1024];
  const int tid = threadIdx.x;
  const unsigned char* bits = args.bits + (long)blockIdx.x * args.n;
  if (tid == 0) v[0] = cmk(1.0, 0.0);
  __syncthreads();
  for (int s = 0; s < args.n; ++s) {
    const int ml = args.dimx[s], mr = args.dimx[s + 1];
    const int b = bits[s] ? 1 : 0;
    const double2* B = args.B[s];
    const int ld = args.ld[s];
    for (int be = tid; be < mr; be += 256) {
      double2 acc = cmk(0.0, 0.0);
      for (int al = 0; al < ml; ++al) acc = cfma(v[al], B[(long)(2 * al + b) * ld + be], acc);
      w[be] = acc;
    }
    __syncthreads();
    for (int be = tid; be < mr; be += 256) v[be] = w[be];
    __syncthreads();
  }
  if (tid == 0) args.out[blockIdx.x] = v[0];
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_prep2(Task2* d_tasks, int ntask, int maxN, hipStream_t st) {
  long nn = (long)maxN * maxN;
  int gx = (int)((nn + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_prep2, dim3(gx, ntask), dim3(256), 0, st, d_tasks);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_theta2(Task2* d_tasks, int ntask, int maxM, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_theta2, dim3((maxM + 63) / 64, (maxN + 63) / 64, ntask), dim3(256), 0, st, d_tasks);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

int jacobi_block_width() { return 8; }

hipError_t launch_jacobi_step(Task2* d_tasks, int ntask, int maxN, int step, int sweep, double tol_mult,
                              int maxin, hipStream_t st) {
  constexpr int BW = 8;
  const int nb = (maxN + BW - 1) / BW;
  const int nbp = nb + (nb & 1);
  hipLaunchKernelGGL(k_jacobi_step<BW>, dim3(nbp / 2, ntask), dim3(256), 0, st, d_tasks, step, sweep,
                     tol_mult, maxin);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_truncate(Task2* d_tasks, int ntask, int chi, double eps, double floor_rel, hipStream_t st) {
  hipLaunchKernelGGL(k_truncate, dim3(ntask), dim3(1024), 0, st, d_tasks, chi, eps, floor_rel);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_split(Task2* d_tasks, int ntask, int maxM, int maxN, int maxK, hipStream_t st) {
  hipLaunchKernelGGL(k_split_right, dim3((maxN + 255) / 256, maxK, ntask), dim3(256), 0, st, d_tasks);
  MPS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_split_left, dim3((maxM + 63) / 64, (maxK + 63) / 64, ntask), dim3(256), 0, st,
                     d_tasks);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_gate1(Task1* d_tasks, int ntask, long maxel, hipStream_t st) {
  int gx = (int)((maxel + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_gate1, dim3(gx, ntask), dim3(256), 0, st, d_tasks);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_amplitude(const AmpArgs& args, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_amplitude, dim3(count), dim3(256), 0, st, args);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
