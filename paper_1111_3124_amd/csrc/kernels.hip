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
#include "gemm.h"

namespace mpsk {

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
//   1. G = A_P^H A_P (W2 x W2, W2 = 2 BW) from the pair's columns A_P of W: row chunks
//      staged in LDS, each wavefront a quarter of the rows, each lane a TB x TB
//      register block of G;
//   2. cyclic two-sided Jacobi on G in LDS, R accumulating the rotations.  Each
//      rotation is the complex symmetric Schur 2x2 (Golub & Van Loan 8.4/8.5) for
//      the pair's Gram entries.  The disjoint pairs of a round act as one unitary J;
//      every thread forms its elements of J^H G J and R J directly from the
//      2x2 neighbourhood of the old values (double-buffered: one barrier a round);
//   3. A_P <- A_P R and V_P <- V_P R (a row per thread), sig2 <- diag(R^H G R).
// A pair whose off-diagonal entries are all below tol * sqrt(G_pp G_qq) is left
// alone; a task whose previous sweep rotated nothing is converged and skipped.
__device__ __forceinline__ int rr_player(int i, int r, int np) { return i == 0 ? 0 : 1 + (i - 1 + r) % (np - 1); }
// partner of index x in round r of the circle schedule on np players
__device__ __forceinline__ int rr_partner(int x, int r, int np) {
  const int pos = x == 0 ? 0 : 1 + ((x - 1 - r) % (np - 1) + (np - 1)) % (np - 1);
  return rr_player(np - 1 - pos, r, np);
}

struct RotCoef {
  double2 al, be;  // (X J)[:, x] = al X[:, x] + be X[:, partner(x)]
  bool rot;
};

// rotation coefficients of index x (partner px) from the current Gram buffer
template <int LD>
__device__ __forceinline__ RotCoef rot_coef(const double2 (*G)[LD], const int* cols, int x, int px, double tol,
                                            double ztol) {
  RotCoef r;
  r.al = cmk(1.0, 0.0);
  r.be = cmk(0.0, 0.0);
  r.rot = false;
  const int p = x < px ? x : px, q = x < px ? px : x;
  if (cols[p] < 0 || cols[q] < 0) return r;
  const double a = G[p][p].x, b = G[q][q].x;
  const double2 g = G[p][q];
  const double ga = hypot(g.x, g.y);
  if (!(a > ztol && b > ztol && ga > tol * sqrt(a * b))) return r;
  const double zeta = (b - a) / (2.0 * ga);
  const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double sn = t * c;
  const double2 e = cmk(g.x / ga, -g.y / ga);  // e^{-i phi}
  r.rot = true;
  if (x == p) { r.al = cmk(c, 0.0); r.be = cscale(e, -sn); }
  else        { r.al = cscale(e, c); r.be = cmk(sn, 0.0); }
  return r;
}

template <int BW>
__global__ __launch_bounds__(256) void k_jacobi_step(Task2* tasks, int step, int sweep, double tol_mult,
                                                      int maxin) {
  constexpr int W2 = 2 * BW;
  constexpr int TB = W2 / 8;          // register block edge of the Gram phase
  constexpr int EPT = (W2 * W2 + 255) / 256;  // inner-phase elements per thread
  static_assert(W2 == 8 || W2 == 16 || W2 == 32, "block width");
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
  __shared__ double2 Gb[2][W2][W2 + 1];
  __shared__ double2 Rb[2][W2][W2 + 1];
  __shared__ int swf[3];
  __shared__ int any_rot;

  const int I = rr_player(pi, step, nbp), J = rr_player(nbp - 1 - pi, step, nbp);
  if (tid < W2) {
    const int blk = tid < BW ? I : J;
    const int c = blk * BW + (tid % BW);
    cols[tid] = (blk < nb && c < N) ? c : -1;
  }
  if (tid < 3) swf[tid] = 0;
  if (tid == 0) any_rot = 0;
  __syncthreads();

  // 1. Gram: wave g takes rows g, g+4, ... of each 64-row chunk; lane (bi, bj) a TB x TB block
  const double2* __restrict__ A = T.thw;
  const int wave = tid >> 6, lane = tid & 63;
  const int bi = lane >> 3, bj = lane & 7;
  double2 acc[TB][TB];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = cmk(0.0, 0.0);
  for (int r0 = 0; r0 < M; r0 += 64) {
    for (int e = tid; e < 64 * W2; e += 256) {
      const int rr = e & 63, l = e >> 6;
      const int c = cols[l], r = r0 + rr;
      Ch[rr][l] = (c >= 0 && r < M) ? A[(long)c * M + r] : cmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = wave; rr < 64; rr += 4) {
      double2 x[TB], y[TB];
#pragma unroll
      for (int i = 0; i < TB; ++i) x[i] = Ch[rr][bi * TB + i];
#pragma unroll
      for (int j = 0; j < TB; ++j) y[j] = Ch[rr][bj * TB + j];
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) acc[i][j] = cfmac(x[i], y[j], acc[i][j]);
    }
    __syncthreads();
  }
  // reduce the four waves' partial Grams into Gb[0] (one wave at a time: deterministic)
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const int gi = bi * TB + i, gj = bj * TB + j;
          if (gi < W2 && gj < W2) Gb[0][gi][gj] = (w == 0) ? acc[i][j] : cadd(Gb[0][gi][gj], acc[i][j]);
        }
    }
    __syncthreads();
  }
  for (int e = tid; e < W2 * W2; e += 256) Rb[0][e / W2][e % W2] = cmk(e / W2 == e % W2 ? 1.0 : 0.0, 0.0);
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-53;
  const double ztol = *T.fro2 * 0x1p-88;  // columns below 2^-44 ||theta|| are rounding noise
  __syncthreads();

  // 2. two-sided Jacobi on G, one barrier per round.  With many column blocks a
  // single inner sweep per step is enough (the next steps revisit every column);
  // with few blocks each pair must be diagonalised fully.
  const int inner = nbp >= 16 ? maxin : 12;
  int cur = 0;
  for (int isw = 0; isw < inner; ++isw) {
    // slot isw%3 is written this sweep and read after its last barrier; slot
    // (isw+1)%3 was last read two sweeps ago (many barriers back): clear it now
    if (tid == 0) swf[(isw + 1) % 3] = 0;
    for (int rnd = 0; rnd < W2 - 1; ++rnd) {
      const double2(*G)[W2 + 1] = Gb[cur];
      const double2(*R)[W2 + 1] = Rb[cur];
      double2 gn[EPT], rn[EPT];
      int ei[EPT], ej[EPT];
      bool any = false;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + 256 * q;
        ei[q] = -1;
        if (e >= W2 * W2) continue;
        const int i = e / W2, j = e % W2;
        ei[q] = i; ej[q] = j;
        const int pi_ = rr_partner(i, rnd, W2), pj = rr_partner(j, rnd, W2);
        const RotCoef ci = rot_coef<W2 + 1>(G, cols, i, pi_, tol, ztol);
        const RotCoef cj = (pj == pi_ && j == i) ? ci : rot_coef<W2 + 1>(G, cols, j, pj, tol, ztol);
        any |= ci.rot;
        // (J^H G J)_{ij} and (R J)_{ij}
        const double2 gij = G[i][j], gipj = G[i][pj], gpij = G[pi_][j], gpipj = G[pi_][pj];
        const double2 colj = cadd(cmul(cj.al, gij), cmul(cj.be, gipj));
        const double2 colpj = cadd(cmul(cj.al, gpij), cmul(cj.be, gpipj));
        double2 v = cadd(cmul(cconj(ci.al), colj), cmul(cconj(ci.be), colpj));
        if (ci.rot && j == pi_) v = cmk(0.0, 0.0);  // the rotated pair's off-diagonal is zero
        if (i == j) v.y = 0.0;
        gn[q] = v;
        rn[q] = cadd(cmul(cj.al, R[i][j]), cmul(cj.be, R[i][pj]));
      }
      if (any) swf[isw % 3] = 1;
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        if (ei[q] >= 0) {
          Gb[cur ^ 1][ei[q]][ej[q]] = gn[q];
          Rb[cur ^ 1][ei[q]][ej[q]] = rn[q];
        }
      cur ^= 1;
      __syncthreads();
    }
    if (!swf[isw % 3]) break;
    if (tid == 0) any_rot = 1;
  }
  __syncthreads();

  // 3. apply R to the pair's columns of W and V
  if (any_rot) {
    const double2(*R)[W2 + 1] = Rb[cur];
    double2* __restrict__ Aw = T.thw;
    double2* __restrict__ Vw = T.V;
    for (int pass = 0; pass < 2; ++pass) {
      double2* X = pass ? Vw : Aw;
      const int rows = pass ? N : M;
      for (int r = tid; r < rows; r += 256) {
        double2 x[W2];
#pragma unroll
        for (int l = 0; l < W2; ++l) x[l] = cols[l] >= 0 ? X[(long)cols[l] * rows + r] : cmk(0.0, 0.0);
#pragma unroll 4
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
  if (tid < W2 && cols[tid] >= 0) T.sig2[cols[tid]] = Gb[cur][tid][tid].x;
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

hipError_t launch_jacobi_step(Task2* d_tasks, int ntask, int maxN, int bw, int step, int sweep, double tol_mult,
                              int maxin, hipStream_t st) {
  const int nb = (maxN + bw - 1) / bw;
  const int nbp = nb + (nb & 1);
  const dim3 grid(nbp / 2, ntask);
  switch (bw) {
    case 4: hipLaunchKernelGGL(k_jacobi_step<4>, grid, dim3(256), 0, st, d_tasks, step, sweep, tol_mult, maxin); break;
    case 8: hipLaunchKernelGGL(k_jacobi_step<8>, grid, dim3(256), 0, st, d_tasks, step, sweep, tol_mult, maxin); break;
    case 16: hipLaunchKernelGGL(k_jacobi_step<16>, grid, dim3(256), 0, st, d_tasks, step, sweep, tol_mult, maxin); break;
    default: return hipErrorInvalidValue;
  }
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
