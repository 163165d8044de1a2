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
// V = I_N, the identity column order, zero the Frobenius accumulator and the
// rotation flags.
__global__ __launch_bounds__(256) void k_prep2(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int N = T.N;
  const long nn = (long)N * N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
    const int r = (int)(e % N), c = (int)(e / N);
    T.V[e] = cmk(r == c ? 1.0 : 0.0, 0.0);
  }
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < N; j += 256) T.perm[j] = j;  // the first sweep's column order
  // no deferred V rotation pending (the workspace may hold another task's data; the
  // tags a task writes grow with its steps, so none of its own can match a later one)
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < 2 * (((N + 7) / 8 + 2) / 2); j += 256) T.VPC[j * 17 + 16] = 0;
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
            if (t->tr)
              t->thw[(long)(2 * al + i) * t->Nt + (j * c_ + ga)] = cconj(ow);
            else
              t->thw[idx] = ow;
          }
      }
    }
  }
};

__global__ __launch_bounds__(256) void k_theta2(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->M || tn >= t->Nt) return;
  ThetaOp op{t};
  cgemm_tile(op, t->M, t->Nt, t->b, tm, tn);
}

// ------------------------------------------------------------------ ||theta_w||_F^2
// Partial sums over fixed chunks of kFroChunk elements of thw (each thread 16 of them
// in order, then a fixed tree), then the partials in chunk order: the result depends
// only on the task, not on the launch.  (thw holds theta_w or its conjugate
// transpose: the same squared magnitudes.)
__global__ __launch_bounds__(256) void k_fro_part(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const long mn = (long)T.M * T.Nt;
  const long c0 = (long)blockIdx.x * kFroChunk;
  if (c0 >= mn) return;
  double s = 0.0;
  for (int q = 0; q < kFroChunk / 256; ++q) {
    const long e = c0 + q * 256 + threadIdx.x;
    if (e < mn) {
      const double2 w = T.thw[e];
      s += w.x * w.x + w.y * w.y;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) T.frop[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_fro_sum(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.x].slot];
  const long mn = (long)T.M * T.Nt;
  const int nch = (int)((mn + kFroChunk - 1) / kFroChunk);
  double s = 0.0;
  for (int c = threadIdx.x; c < nch; c += 256) s += T.frop[c];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *T.fro2 = red[0];
}

// ------------------------------------------------------------------ Jacobi step
// One step of the block one-sided Jacobi sweep.  Columns are grouped in blocks of
// BW; the blocks are paired by the round-robin ("circle") schedule, so that the
// 2*BW-column groups of one step are disjoint and all block pairs meet once per
// sweep.  Each 512-thread block takes one pair of one task:
//   1. G = A_P^H A_P (W2 x W2, W2 = 2 BW) from the pair's columns A_P of W: row chunks
//      staged in LDS, each wavefront an eighth of the rows, each lane a TB x TB
//      register block of G;
//   2. two-sided Jacobi on G in LDS, R accumulating the rotations.  Each rotation is
//      the complex symmetric Schur 2x2 (Golub & Van Loan 8.4/8.5) for the pair's
//      Gram entries.  The disjoint pairs of a round act as one unitary J; every
//      thread forms its elements of J^H G J and R J directly from the 2x2
//      neighbourhood of the old values (double-buffered).  With many blocks, a
//      block's inner pairs are rotated at the sweep's first step and the later
//      steps rotate only the pairs across the two blocks (BW rounds, not 2 BW - 1);
//   3. A_P <- A_P R and V_P <- V_P R (16-column pairs: half the rows in tiles of 16 on
//      the matrix cores, half on the vector units; other widths: a row per thread),
//      sig2 <- diag(R^H G R).
// A pair whose off-diagonal entries are all below tol * sqrt(G_pp G_qq) is left
// alone; a task whose previous sweep rotated nothing is converged and skipped.
__device__ __forceinline__ int rr_player(int i, int r, int np) { return i == 0 ? 0 : 1 + (i - 1 + r) % (np - 1); }
// accumulator of v_mfma_f64_16x16x4f64: element r of lane l is D[l / 16 + 4 r][l % 16]
// (A operand: lane l holds A[l % 16][l / 16]; B operand: B[l / 16][l % 16])
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
// Newton-refined reciprocal square root (the hardware estimate v_rsq_f64 is not
// correctly rounded; two Newton steps bring it to binary64 accuracy, with a much
// shorter dependency chain than div / sqrt).
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Block-wide inner two-sided Jacobi on the pair's W2 x W2 Gram (NT threads).  Per
// round every thread takes elements (i, j): it forms the rotations of i's and of j's
// pair itself from the old G (each pair's rotation is computed identically by every
// thread that needs it), then its elements of J^H G J and R J from the 2 x 2
// neighbourhood of the old values (double-buffered): one barrier a round.  G[0] holds
// the Gram on entry; returns the buffer with the result; any_rot is set when
// something rotated.
template <int W2>
struct InnerLds {
  int any_rot;
};

// Partner of column x in an inner round: cross rounds pair x < H with H + (x + rnd)
// mod H; the full round-robin holds column 0 at position 0 and column x > 0 at
// position 1 + (x - 1 - rnd) mod (W2 - 1), position k meeting W2 - 1 - k.
//
// Branch-free (selects only, so that a round is one basic block the compiler can
// schedule as a whole): rnd < W2 - 1 and H a power of two keep every intermediate
// within one period.
template <int W2>
__device__ __forceinline__ int inner_partner(int x, int rnd, bool cross) {
  constexpr int H = W2 / 2, np1 = W2 - 1;
  static_assert((H & (H - 1)) == 0, "H a power of two");
  const bool lo = x < H;
  const int pc = ((x + (lo ? rnd : -rnd)) & (H - 1)) + (lo ? H : 0);
  int v = x - 1 - rnd;
  v = v < 0 ? v + np1 : v;
  const int m = np1 - (x == 0 ? 0 : 1 + v);  // the partner's position
  int q = m - 1 + rnd;
  q = q >= np1 ? q - np1 : q;
  const int pf = m == 0 ? 0 : 1 + q;
  return cross ? pc : pf;
}

// Rotation of one column pair (p < q) from the Gram entries al = G_pp, be = G_qq,
// g = G_pq: the complex form of the symmetric Schur 2x2 (Golub & Van Loan 8.4):
// with e = conj(g)/|g|, zeta = (be - al) / (2|g|), t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = t c:  (X J)[:, p] = c X_p - s e X_q,  (X J)[:, q] = s X_p + c e X_q.
// With u = |zeta| + sqrt(1 + zeta^2) = 1 / |t|, c = u / sqrt(u^2 + 1) and |s| = 1 / sqrt(u^2 + 1),
// which needs no reciprocal; sqrt(x) for x >= 1 is x rsq(x).  A pair is rotated when
// both columns are above the zero threshold ztol and |g|^2 > tol^2 G_pp G_qq.
//
// Column x's coefficients in the round's unitary J, (X J)[:, x] = ra X_x + rb X_px,
// from its pair's Gram entries al = G_pp, be = G_qq, g = G_pq (p < q) and whether x
// is p.  Branch-free: the rotation is formed whether or not the pair rotates (the
// operands are all loaded before), then selected; the same inputs give every thread
// that needs the pair the same rotation.
struct RotCoef {
  double2 ra, rb;
  int rot;
};

__device__ __forceinline__ RotCoef inner_coef(double al, double be, double2 g, bool valid, bool xp, double tol,
                                              double ztol) {
  const double g2 = g.x * g.x + g.y * g.y;
  const bool rot = valid & (al > ztol) & (be > ztol) & (g2 > tol * tol * al * be);
  const double ig = rsq_nr(g2);  // 1 / |g|
  const double zeta = 0.5 * (be - al) * ig;
  const double x = fma(zeta, zeta, 1.0);
  const double u = fabs(zeta) + x * rsq_nr(x);
  const double w = rsq_nr(fma(u, u, 1.0));
  const double c = u * w, sn = zeta < 0.0 ? -w : w;
  const double ex = g.x * ig, ey = -g.y * ig;
  // every candidate formed, then selected component by component (no branches)
  const double cex = ex * c, cey = ey * c, sex = ex * -sn, sey = ey * -sn;
  RotCoef k;
  k.rot = rot ? 1 : 0;
  k.ra.x = rot ? (xp ? c : cex) : 1.0;
  k.ra.y = rot ? (xp ? 0.0 : cey) : 0.0;
  k.rb.x = rot ? (xp ? sex : sn) : 0.0;
  k.rb.y = rot ? (xp ? sey : 0.0) : 0.0;
  return k;
}

// The same inner Jacobi for wide pairs (W2 = 32), organised by pairs: each round,
// one thread per column pair forms both columns' coefficients (staged in LDS), then
// one thread per pair of pairs (a, b) forms the 2 x 2 blocks of J^H G J and R J on
// rows {p_a, q_a} and columns {p_b, q_b}, which need only that block of G and R.
// Every coefficient comes from the same inputs through the same inner_coef as in
// inner_jacobi_block and every element from the same expression, so both forms give
// the same G and R bit for bit; this one reads each G and R element once a round.
template <int W2>
struct StagedRot {
  double2 ra[W2], rb[W2];
  int rot[W2];
};

// the columns (p < q) of pair a in round rnd: cross rounds pair a < W2/2 with
// W2/2 + (a + rnd) mod W2/2; the full round-robin pairs positions a and W2 - 1 - a,
// position 0 holding column 0 and position m > 0 column 1 + (m - 1 + rnd) mod (W2 - 1)
template <int W2>
__device__ __forceinline__ void inner_pair(int a, int rnd, bool cross, int& p, int& q) {
  constexpr int H = W2 / 2, np1 = W2 - 1;
  if (cross) {
    p = a;
    q = H + (a + rnd) % H;
    return;
  }
  const int m0 = a, m1 = np1 - a;
  const int c0 = m0 == 0 ? 0 : 1 + (m0 - 1 + rnd) % np1, c1 = 1 + (m1 - 1 + rnd) % np1;
  p = c0 < c1 ? c0 : c1;
  q = c0 < c1 ? c1 : c0;
}

template <int W2, int NT>
__device__ int inner_jacobi_pairs(double2 (&G)[2][W2][W2 + 1], double2 (&R)[2][W2][W2 + 1], InnerLds<W2>& L,
                                  StagedRot<W2>& K, const int (&cols)[W2], int inner, double tol, double ztol,
                                  bool cross) {
  constexpr int H = W2 / 2;
  static_assert(NT >= H * H, "one thread per pair of pairs");
  const int tid = threadIdx.x;
  for (int e = tid; e < W2 * W2; e += NT) R[0][e / W2][e % W2] = cmk(e / W2 == e % W2 ? 1.0 : 0.0, 0.0);
  __syncthreads();
  int cur = 0, any_rot = 0;
  const int nrnd = cross ? H : W2 - 1;
  for (int isw = 0; isw < inner; ++isw) {
    int mine = 0;
    for (int rnd = 0; rnd < nrnd; ++rnd) {
      const double2(*Gc)[W2 + 1] = G[cur];
      if (tid < H) {  // pair tid's rotation: coefficients of both columns
        int p, q;
        inner_pair<W2>(tid, rnd, cross, p, q);
        const bool v = (cols[p] >= 0) & (cols[q] >= 0);
        const double al = Gc[p][p].x, be = Gc[q][q].x;
        const double2 g = Gc[p][q];
        const RotCoef cp = inner_coef(al, be, g, v, true, tol, ztol);
        const RotCoef cq = inner_coef(al, be, g, v, false, tol, ztol);
        K.ra[p] = cp.ra;
        K.rb[p] = cp.rb;
        K.rot[p] = cp.rot;
        K.ra[q] = cq.ra;
        K.rb[q] = cq.rb;
        K.rot[q] = cq.rot;
        mine |= cp.rot;
      }
      __syncthreads();
      if (tid < H * H) {
        int pa, qa, pb, qb;
        inner_pair<W2>(tid / H, rnd, cross, pa, qa);
        inner_pair<W2>(tid % H, rnd, cross, pb, qb);
        const double2 g_pp = Gc[pa][pb], g_pq = Gc[pa][qb], g_qp = Gc[qa][pb], g_qq = Gc[qa][qb];
        const double2 r_pp = R[cur][pa][pb], r_pq = R[cur][pa][qb], r_qp = R[cur][qa][pb], r_qq = R[cur][qa][qb];
        const double2 ra_pa = K.ra[pa], rb_pa = K.rb[pa], ra_qa = K.ra[qa], rb_qa = K.rb[qa];
        const double2 ra_pb = K.ra[pb], rb_pb = K.rb[pb], ra_qb = K.ra[qb], rb_qb = K.rb[qb];
        const int rot_pa = K.rot[pa], rot_qa = K.rot[qa];
        // element (i, j) with partners (pi, pj): from G[i][j], G[i][pj], G[pi][j], G[pi][pj]
        auto elem = [&](int i, int j, int pi_, double2 ra_i, double2 rb_i, int rot_i, double2 ra_j, double2 rb_j,
                        double2 gij, double2 giq, double2 gpj, double2 gpq) {
          const double2 colj = cadd(cmul(ra_j, gij), cmul(rb_j, giq));
          const double2 colpj = cadd(cmul(ra_j, gpj), cmul(rb_j, gpq));
          double2 v = cadd(cmul(cconj(ra_i), colj), cmul(cconj(rb_i), colpj));
          if (rot_i && j == pi_) v = cmk(0.0, 0.0);  // the rotated pair's off-diagonal is zero
          if (i == j) v.y = 0.0;
          return v;
        };
        double2(*Gn)[W2 + 1] = G[cur ^ 1];
        double2(*Rn)[W2 + 1] = R[cur ^ 1];
        Gn[pa][pb] = elem(pa, pb, qa, ra_pa, rb_pa, rot_pa, ra_pb, rb_pb, g_pp, g_pq, g_qp, g_qq);
        Gn[pa][qb] = elem(pa, qb, qa, ra_pa, rb_pa, rot_pa, ra_qb, rb_qb, g_pq, g_pp, g_qq, g_qp);
        Gn[qa][pb] = elem(qa, pb, pa, ra_qa, rb_qa, rot_qa, ra_pb, rb_pb, g_qp, g_qq, g_pp, g_pq);
        Gn[qa][qb] = elem(qa, qb, pa, ra_qa, rb_qa, rot_qa, ra_qb, rb_qb, g_qq, g_qp, g_pq, g_pp);
        Rn[pa][pb] = cadd(cmul(ra_pb, r_pp), cmul(rb_pb, r_pq));
        Rn[pa][qb] = cadd(cmul(ra_qb, r_pq), cmul(rb_qb, r_pp));
        Rn[qa][pb] = cadd(cmul(ra_pb, r_qp), cmul(rb_pb, r_qq));
        Rn[qa][qb] = cadd(cmul(ra_qb, r_qq), cmul(rb_qb, r_qp));
      }
      cur ^= 1;
      __syncthreads();
    }
    if (!__syncthreads_or(mine)) break;
    any_rot = 1;
  }
  if (tid == 0) L.any_rot = any_rot;
  __syncthreads();
  return cur;
}

// cross: only the (W2/2)^2 pairs between the two column blocks, in W2/2 rounds
// (round r pairs p with W2/2 + (p + r) mod W2/2); else all pairs, round-robin.
template <int W2, int NT>
__device__ int inner_jacobi_block(double2 (&G)[2][W2][W2 + 1], double2 (&R)[2][W2][W2 + 1], InnerLds<W2>& L,
                                  const int (&cols)[W2], int inner, double tol, double ztol, bool cross = false) {
  const int tid = threadIdx.x;
  for (int e = tid; e < W2 * W2; e += NT) R[0][e / W2][e % W2] = cmk(e / W2 == e % W2 ? 1.0 : 0.0, 0.0);
  __syncthreads();
  int cur = 0, any_rot = 0;
  const int nrnd = cross ? W2 / 2 : W2 - 1;
  for (int isw = 0; isw < inner; ++isw) {
    int mine = 0;  // did a pair this thread used rotate in this inner sweep
    for (int rnd = 0; rnd < nrnd; ++rnd) {
      for (int e = tid; e < W2 * W2; e += NT) {
        const int i = e / W2, j = e % W2;
        const int pi_ = inner_partner<W2>(i, rnd, cross), pj = inner_partner<W2>(j, rnd, cross);
        const bool ip = i < pi_, jp = j < pj;
        const double2(*Gc)[W2 + 1] = G[cur];
        // every operand of the round first (one LDS round trip)
        const bool vi = (cols[i] >= 0) & (cols[pi_] >= 0), vj = (cols[j] >= 0) & (cols[pj] >= 0);
        const double gii = Gc[i][i].x, gpp = Gc[pi_][pi_].x, gjj = Gc[j][j].x, gqq = Gc[pj][pj].x;
        const double2 gi = ip ? Gc[i][pi_] : Gc[pi_][i], gj = jp ? Gc[j][pj] : Gc[pj][j];
        const double2 g_ij = Gc[i][j], g_iq = Gc[i][pj], g_pj = Gc[pi_][j], g_pq = Gc[pi_][pj];
        const double2 r_ij = R[cur][i][j], r_iq = R[cur][i][pj];
        const RotCoef ci = inner_coef(ip ? gii : gpp, ip ? gpp : gii, gi, vi, ip, tol, ztol);
        const RotCoef cj = inner_coef(jp ? gjj : gqq, jp ? gqq : gjj, gj, vj, jp, tol, ztol);
        mine |= ci.rot | cj.rot;
        const double2 colj = cadd(cmul(cj.ra, g_ij), cmul(cj.rb, g_iq));
        const double2 colpj = cadd(cmul(cj.ra, g_pj), cmul(cj.rb, g_pq));
        double2 v = cadd(cmul(cconj(ci.ra), colj), cmul(cconj(ci.rb), colpj));
        if (ci.rot && j == pi_) v = cmk(0.0, 0.0);  // the rotated pair's off-diagonal is zero
        if (i == j) v.y = 0.0;
        G[cur ^ 1][i][j] = v;
        R[cur ^ 1][i][j] = cadd(cmul(cj.ra, r_ij), cmul(cj.rb, r_iq));
      }
      cur ^= 1;
      __syncthreads();  // (a round that rotated nothing copied G and R unchanged)
    }
    if (!__syncthreads_or(mine)) break;
    any_rot = 1;
  }
  if (tid == 0) L.any_rot = any_rot;
  __syncthreads();
  return cur;
}

// The same inner Jacobi with each column's coefficients formed once a round: W2
// threads form them (column x from its pair's Gram entries, as in inner_jacobi_block)
// and stage them in LDS; after a barrier every thread forms one element, of J^H G J
// (the first W2^2 threads) or of R J (the next W2^2), from the staged coefficients by
// the expressions of inner_jacobi_block.  Two barriers a round, but no thread forms a
// rotation twice and the elements spread over all the block's waves.  The fused and
// the split step both use it for 16-column pairs, so they form the same G and R.
template <int W2, int NT>
__device__ int inner_jacobi_staged(double2 (&G)[2][W2][W2 + 1], double2 (&R)[2][W2][W2 + 1], InnerLds<W2>& L,
                                   StagedRot<W2>& K, const int (&cols)[W2], int inner, double tol, double ztol,
                                   bool cross) {
  constexpr int E = W2 * W2;
  static_assert(NT >= W2, "one thread per column");
  const int tid = threadIdx.x;
  for (int e = tid; e < E; e += NT) R[0][e / W2][e % W2] = cmk(e / W2 == e % W2 ? 1.0 : 0.0, 0.0);
  __syncthreads();
  int cur = 0, any_rot = 0;
  const int nrnd = cross ? W2 / 2 : W2 - 1;
  for (int isw = 0; isw < inner; ++isw) {
    int mine = 0;
    for (int rnd = 0; rnd < nrnd; ++rnd) {
      const double2(*Gc)[W2 + 1] = G[cur];
      if (tid < W2) {  // column tid's coefficients in this round's unitary
        const int x = tid, px = inner_partner<W2>(x, rnd, cross);
        const bool xp = x < px;
        const int p = xp ? x : px, q = xp ? px : x;
        const bool v = (cols[x] >= 0) & (cols[px] >= 0);
        const RotCoef c = inner_coef(Gc[p][p].x, Gc[q][q].x, Gc[p][q], v, xp, tol, ztol);
        K.ra[x] = c.ra;
        K.rb[x] = c.rb;
        K.rot[x] = c.rot;
        mine |= c.rot;
      }
      __syncthreads();
      for (int e = tid; e < 2 * E; e += NT) {
        const bool isG = e < E;
        const int i = (e % E) / W2, j = e % W2;
        const int pi_ = inner_partner<W2>(i, rnd, cross), pj = inner_partner<W2>(j, rnd, cross);
        const double2 ra_j = K.ra[j], rb_j = K.rb[j];
        if (isG) {
          const double2 ra_i = K.ra[i], rb_i = K.rb[i];
          const int rot_i = K.rot[i];
          const double2 g_ij = Gc[i][j], g_iq = Gc[i][pj], g_pj = Gc[pi_][j], g_pq = Gc[pi_][pj];
          const double2 colj = cadd(cmul(ra_j, g_ij), cmul(rb_j, g_iq));
          const double2 colpj = cadd(cmul(ra_j, g_pj), cmul(rb_j, g_pq));
          double2 v = cadd(cmul(cconj(ra_i), colj), cmul(cconj(rb_i), colpj));
          if (rot_i && j == pi_) v = cmk(0.0, 0.0);  // the rotated pair's off-diagonal is zero
          if (i == j) v.y = 0.0;
          G[cur ^ 1][i][j] = v;
        } else {
          R[cur ^ 1][i][j] = cadd(cmul(ra_j, R[cur][i][j]), cmul(rb_j, R[cur][i][pj]));
        }
      }
      cur ^= 1;
      __syncthreads();
    }
    if (!__syncthreads_or(mine)) break;
    any_rot = 1;
  }
  if (tid == 0) L.any_rot = any_rot;
  __syncthreads();
  return cur;
}

// A_P <- A_P R (and V_P <- V_P R) for 16-column pairs, split between the two FP64
// pipelines, whose peaks are equal: the first half of each matrix's 16-row tiles on
// the matrix cores (rot_tiles), its remaining rows on the vector units (rot_rows), in
// different waves so that both issue at once (RotSet below).  Each row is formed by
// the same instructions wherever it is computed, so the fused and split steps give the
// same rows bit for bit.
//
// rot_tiles: per tile Y^T = R^T X^T as four k-steps of v_mfma_f64_16x16x4f64 over the
// pair's columns, complex as
//   Re Y^T = Re R^T Re X^T - Im R^T Im X^T,   Im Y^T = Im R^T Re X^T + Re R^T Im X^T.
// R^T is the A operand (k-step s: lane l holds R[4 s + l / 16][l % 16]), loaded from LDS
// once a block; X^T the B operand (lane l holds X[row0 + l % 16][column 4 s + l / 16]);
// element r of lane l's result is Y[row0 + l % 16][column l / 16 + 4 r].  Each element
// of X is loaded and stored by the same lane, so the update is in place.  R's rows and
// columns for absent columns (cols < 0) are the identity's and their loads read zero.
struct RotA {
  double re[4], im[4];
};

__device__ __forceinline__ RotA rot_operand(const double2 (*R)[17], int lane) {
  RotA a;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 v = R[4 * s + (lane >> 4)][lane & 15];
    a.re[s] = v.x;
    a.im[s] = v.y;
  }
  return a;
}

// The rows an update rotates: W (Mw rows) and V (Nv rows; either may be absent, with 0
// rows).  Each matrix's first half of 16-row tiles (hw, hv tiles) goes to the matrix
// cores, its remaining rows to the vector units, wherever it is updated, so every row
// is formed by the same instructions in the fused step, the split step and the
// deferred V update.  The matrix-core part is indexed as W's tiles, then V's; the
// vector part as W's remaining rows, then V's.
struct RotSet {
  double2* W;
  double2* V;
  int Mw, Nv, hw, hv;
};
__device__ __forceinline__ RotSet rot_set(double2* W, int Mw, double2* V, int Nv) {
  return RotSet{W, V, Mw, Nv, ((Mw + 15) / 16 + 1) / 2, ((Nv + 15) / 16 + 1) / 2};
}

// matrix-core tiles t0, t0 + stride, ... below hw + hv, four a group: the group's loads
// first, then each tile's products and stores
__device__ __forceinline__ void rot_tiles(const RotSet& S, int t0, int stride, const int (&cols)[16], const RotA& a,
                                          int lane) {
  constexpr int G = 4;
  const int j = lane & 15, kq = lane >> 4, t1 = S.hw + S.hv;
  for (int t = t0; t < t1; t += G * stride) {
    double2 x[G][4];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int tt = t + u * stride;
      const bool inW = tt < S.hw;
      double2* X = inW ? S.W : S.V;
      const int rows = inW ? S.Mw : S.Nv, r = 16 * (inW ? tt : tt - S.hw) + j;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int c = cols[4 * s + kq];
        x[u][s] = (tt < t1 && c >= 0 && r < rows) ? X[(long)c * rows + r] : cmk(0.0, 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int tt = t + u * stride;
      if (tt >= t1) break;
      mfma_d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re[s], x[u][s].x, yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im[s], x[u][s].x, yi, 0, 0, 0);
        yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im[s], -x[u][s].y, yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re[s], x[u][s].y, yi, 0, 0, 0);
      }
      const bool inW = tt < S.hw;
      double2* X = inW ? S.W : S.V;
      const int rows = inW ? S.Mw : S.Nv, r = 16 * (inW ? tt : tt - S.hw) + j;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cols[kq + 4 * q];
        // recomputed, not kept from the loads (16 live 64-bit addresses would cost
        // the block its second slot on the CU)
        long off = (long)c * rows + r;
        __asm__ volatile("" : "+v"(off));
        if (c >= 0 && r < rows) X[off] = cmk(yr[q], yi[q]);
      }
    }
  }
}

// the vector units' rows, one a thread (threads i0, i0 + nth, ...): the row times R
__device__ __forceinline__ void rot_rows(const RotSet& S, int i0, int nth, const int (&cols)[16],
                                         const double2 (*R)[17]) {
  const int rw = S.Mw > 16 * S.hw ? S.Mw - 16 * S.hw : 0, rv = S.Nv > 16 * S.hv ? S.Nv - 16 * S.hv : 0;
  for (int e = i0; e < rw + rv; e += nth) {
    const bool inW = e < rw;
    double2* X = inW ? S.W : S.V;
    const int rows = inW ? S.Mw : S.Nv, r = inW ? 16 * S.hw + e : 16 * S.hv + e - rw;
    double2 x[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) x[l] = cols[l] >= 0 ? X[(long)cols[l] * rows + r] : cmk(0.0, 0.0);
#pragma unroll 4
    for (int pc = 0; pc < 16; ++pc) {
      double2 y = cmk(0.0, 0.0);
#pragma unroll
      for (int l = 0; l < 16; ++l) y = cfma(x[l], R[l][pc], y);
      if (cols[pc] >= 0) X[(long)cols[pc] * rows + r] = y;
    }
  }
}

// the set's update by a whole 512-thread block: matrix-core part by waves 0-3, vector
// part by waves 4-7
__device__ __forceinline__ void rot_update(const RotSet& S, const int (&cols)[16], const double2 (*R)[17]) {
  const int tid = threadIdx.x;
  if (tid < 256)
    rot_tiles(S, tid >> 6, 4, cols, rot_operand(R, tid & 63), tid & 63);
  else
    rot_rows(S, tid - 256, 256, cols, R);
}

// entry of Task2::VPR / VPC written by pair `pair` at global step g (two step parities
// of ((N + 7) / 8 + 2) / 2 pairs each, enough for the padded block count)
__device__ __forceinline__ long vp_entry(int N, int g, int pair) {
  return (long)(g & 1) * (((N + 7) / 8 + 2) / 2) + pair;
}

// V's deferred rotation of pair pv at global step g (see Task2::VPR): the rotation
// the pair's block stored at step g - 1, applied to V if its tag says so, then marked
// as applied.  A whole 512-thread block; R and cols staged in LDS.
__device__ __forceinline__ void apply_deferred_v(const Task2& T, int pv, int g, double2 (*R)[17], int (&cols)[16]) {
  const int tid = threadIdx.x;
  if (g < 1) return;
  const long e = vp_entry(T.N, g - 1, pv);
  int* c = T.VPC + e * 17;
  // the entry's columns and R loaded together with its tag (one memory latency, not
  // two; the entry lies in the task's workspace whatever the tag says)
  const int cl = tid < 16 ? c[tid] : 0;
  const double2 rv = tid < 256 ? T.VPR[e * 256 + tid] : cmk(0.0, 0.0);
  if (c[16] != g) return;  // (uniform: every thread reads the same tag)
  if (tid < 16) cols[tid] = cl;
  if (tid < 256) R[tid / 16][tid % 16] = rv;
  __syncthreads();
  rot_update(rot_set(nullptr, 0, T.JV, T.N), cols, R);
  __syncthreads();
  if (tid == 0) c[16] = 0;
}

// One Jacobi step: blockIdx.x is a column-block pair (I, J) of the round-robin
// schedule, blockIdx.y a task; 512 threads.  Rotating the pair's 2 BW columns:
//   1. G = A_P^H A_P (W2 x W2, A_P = the pair's columns of W) from row chunks staged
//      in LDS, D chunks of loads in flight;
//   2. inner two-sided Jacobi on G (inner_jacobi_block), R accumulating the rotations;
//   3. A_P <- A_P R and V_P <- V_P R (16-column pairs: rot_tiles and rot_rows side by
//      side; other widths: a row a thread), sig2 <- diag(R^H G R).
//   Block width 8: V_P's update waits one step.  The pair's block stores R, and a
//   second set of blocks in the grid, one a pair (`defer`: the host sets it for every
//   launch that holds a task accumulating V), applies the previous step's stored
//   rotations to V while the pairs' blocks run; a flush applies the last step's.  V's
//   rows are formed by the same instructions as in the split step, which updates V at
//   once.
template <int BW>
__global__ __launch_bounds__(512) void k_jacobi_step(Task2* tasks, const Ent* ents, int step, double tol_mult,
                                                        int maxin, int maxin_few, int defer, long long* phase_clock) {
  constexpr int NT = 512, NW = NT / 64;
  constexpr int W2 = 2 * BW;
  constexpr int TB = W2 / 8;
  constexpr int CR = 1024 / W2;                // rows per Gram chunk
  constexpr int LPT = CR * W2 / NT;            // chunk elements loaded per thread
  constexpr int D = 4;                         // chunks in flight
  constexpr int RPT = 1;                       // update: rows a thread per pass
  static_assert(W2 == 8 || W2 == 16 || W2 == 32, "block width");
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int sweep = ents[blockIdx.y].sweep;
  const int N = T.N, M = T.JR;
  const int nb = (N + BW - 1) / BW;
  const int nbp = nb + (nb & 1);
  const int tid = threadIdx.x;
  __shared__ int cols[W2];
  __shared__ double2 Gb[2][W2][W2 + 1];
  __shared__ double2 Rb[2][W2][W2 + 1];
  __shared__ InnerLds<W2> L;
  if constexpr (W2 == 16) {
    if (defer && (int)blockIdx.x >= (int)gridDim.x / 2) {  // V's rotations of the previous step
      const int pv = blockIdx.x - gridDim.x / 2;
      if (T.jvec && pv < nbp / 2) apply_deferred_v(T, pv, sweep * (nbp - 1) + min(step, nbp - 1), Rb[0], cols);
      return;
    }
  }
  const int pi = blockIdx.x;
  if (step >= nbp - 1 || pi >= nbp / 2) return;
  int* flags = T.flags;
  // slot (sweep+1)%3 is neither read nor written during this sweep: clear it for the
  // next one (also for converged tasks, whose later sweeps must read 0)
  if (step == 0 && pi == 0 && tid == 0) flags[(sweep + 1) % 3] = 0;
  if (sweep > 0 && flags[(sweep + 2) % 3] == 0) return;

  const bool clk = phase_clock && pi == 0 && blockIdx.y == 0 && tid == 0;
  if (clk) phase_clock[0] = wall_clock64();
  // loaded here, so that its latency under the memory phases' traffic is hidden
  const double fro2 = *T.fro2;
  const int I = rr_player(pi, step, nbp), J = rr_player(nbp - 1 - pi, step, nbp);
  if (tid < W2) {  // the pair's columns: positions blk * BW + x of this sweep's order
    const int blk = tid < BW ? I : J;
    const int c = blk * BW + (tid % BW);
    cols[tid] = (blk < nb && c < N) ? T.perm[c] : -1;
  }
  __syncthreads();

  // 1. Gram
  const double2* __restrict__ A = T.JW;
  const int wave = tid >> 6, lane = tid & 63;
  if constexpr (W2 == 16) {
    // by MFMA over k-steps of 4 rows: waves 0-3 take the first half of the rows,
    // waves 4-7 the second, wave w of a half its k-steps w, w + 4, ... (exactly as the
    // blocks of the split step, so both forms give the same G bit for bit); lane l
    // holds X[4 ks + l / 16][column l % 16], the same element for both operands;
    // Re G = Xr^T Xr + Xi^T Xi and, with P = Xr^T Xi, Im G = P - P^T
    static_assert(NW == 8, "two halves of four waves");
    __shared__ double Gw[NW][2][W2][W2 + 1];
    constexpr int KB = 16;  // k-steps of loads in flight per wave
    mfma_d4 gr = {0.0, 0.0, 0.0, 0.0}, gp = {0.0, 0.0, 0.0, 0.0};
    const int c = cols[lane & 15];
    const int roff = lane >> 4;
    const int hh = wave >> 2, wl = wave & 3;
    const int Mh = (M + 1) / 2;
    const int r_lo = hh * Mh, r_hi = min(M, r_lo + Mh);
    const int nks = (r_hi - r_lo + 3) / 4;
    for (int ks0 = wl; ks0 < nks; ks0 += 4 * KB) {
      double2 x[KB];
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        const int r = r_lo + (ks0 + 4 * t) * 4 + roff;
        x[t] = (c >= 0 && r < r_hi) ? A[(long)c * M + r] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        gr = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].x, x[t].x, gr, 0, 0, 0);
        gr = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].y, x[t].y, gr, 0, 0, 0);
        gp = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].x, x[t].y, gp, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Gw[wave][0][roff + 4 * r][lane & 15] = gr[r];
      Gw[wave][1][roff + 4 * r][lane & 15] = gp[r];
    }
    __syncthreads();
    if (tid < W2 * W2) {  // each half's sums in wave order, then the two halves
      const int i = tid / W2, j = tid % W2;
      double sr[2], pij[2], pji[2];
      for (int h = 0; h < 2; ++h) {
        sr[h] = pij[h] = pji[h] = 0.0;
        for (int w = 4 * h; w < 4 * h + 4; ++w) {
          sr[h] += Gw[w][0][i][j];
          pij[h] += Gw[w][1][i][j];
          pji[h] += Gw[w][1][j][i];
        }
      }
      Gb[0][i][j] = cmk(sr[0] + sr[1], (pij[0] + pij[1]) - (pji[0] + pji[1]));
    }
  } else if constexpr (W2 == 32) {
    // by MFMA, the pair's 32 columns as two halves of 16: per k-step of 4 rows lane l
    // holds X[4 ks + l / 16][l % 16] of each half (x0, x1).  Re G = Xr^T Xr + Xi^T Xi
    // from the tiles 00, 01 and 11 (10 = 01^T), P = Xr^T Xi from all four tiles, then
    // Im G = P - P^T; wave w takes the k-steps w, w + 8, ...; the waves' tiles are
    // summed by a fixed tree ((w0 + w1) + (w2 + w3)) + ((w4 + w5) + (w6 + w7)).
    __shared__ double Gs[2][W2][W2 + 1];
    __shared__ double Gx[NW / 2][7][4][64];
    constexpr int KB = 8;  // k-steps of loads in flight per wave
    mfma_d4 t[7];  // Re 00, 01, 11; P 00, 01, 10, 11
#pragma unroll
    for (int k = 0; k < 7; ++k) t[k] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    const int c0 = cols[lane & 15], c1 = cols[16 + (lane & 15)];
    const int roff = lane >> 4;
    const int nks = (M + 3) / 4;
    for (int ks0 = wave; ks0 < nks; ks0 += NW * KB) {
      double2 x0[KB], x1[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int r = (ks0 + NW * u) * 4 + roff;
        x0[u] = (c0 >= 0 && r < M) ? A[(long)c0 * M + r] : cmk(0.0, 0.0);
        x1[u] = (c1 >= 0 && r < M) ? A[(long)c1 * M + r] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        t[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].x, x0[u].x, t[0], 0, 0, 0);
        t[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].y, x0[u].y, t[0], 0, 0, 0);
        t[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].x, x1[u].x, t[1], 0, 0, 0);
        t[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].y, x1[u].y, t[1], 0, 0, 0);
        t[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u].x, x1[u].x, t[2], 0, 0, 0);
        t[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u].y, x1[u].y, t[2], 0, 0, 0);
        t[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].x, x0[u].y, t[3], 0, 0, 0);
        t[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u].x, x1[u].y, t[4], 0, 0, 0);
        t[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u].x, x0[u].y, t[5], 0, 0, 0);
        t[6] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u].x, x1[u].y, t[6], 0, 0, 0);
      }
    }
    for (int stride = 1; stride < NW; stride <<= 1) {
      const int sl = wave / (2 * stride), pos = wave & (2 * stride - 1);
      if (pos == stride) {
#pragma unroll
        for (int k = 0; k < 7; ++k)
#pragma unroll
          for (int r = 0; r < 4; ++r) Gx[sl][k][r][lane] = t[k][r];
      }
      __syncthreads();
      if (pos == 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k)
#pragma unroll
          for (int r = 0; r < 4; ++r) t[k][r] += Gx[sl][k][r][lane];
      }
      __syncthreads();
    }
    if (wave == 0) {
      const int j = lane & 15;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = roff + 4 * r;
        Gs[0][i][j] = t[0][r];
        Gs[0][i][16 + j] = t[1][r];
        Gs[0][16 + i][16 + j] = t[2][r];
        Gs[1][i][j] = t[3][r];
        Gs[1][i][16 + j] = t[4][r];
        Gs[1][16 + i][j] = t[5][r];
        Gs[1][16 + i][16 + j] = t[6][r];
      }
    }
    __syncthreads();
    for (int e = tid; e < W2 * W2; e += NT) {
      const int i = e / W2, j = e % W2;
      // Re G's lower-left tile is the transpose of its upper-right one
      const double re = (i >= 16 && j < 16) ? Gs[0][j][i] : Gs[0][i][j];
      Gb[0][i][j] = cmk(re, Gs[1][i][j] - Gs[1][j][i]);
    }
  } else {
    // row chunks staged in LDS, D chunks of loads in flight; each wave an eighth of
    // a chunk's rows, each lane a TB x TB register block of G
    __shared__ double2 Ch[2][CR][W2 + 1];
    auto load_chunk = [&](int r0, double2 (&v)[LPT]) {
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int e = tid + NT * q;
        const int c = cols[e / CR], r = r0 + e % CR;
        v[q] = (c >= 0 && r < M) ? A[(long)c * M + r] : cmk(0.0, 0.0);
      }
    };
    const int bi = lane >> 3, bj = lane & 7;
    double2 acc[TB][TB];
#pragma unroll
    for (int i = 0; i < TB; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j) acc[i][j] = cmk(0.0, 0.0);
    const int nch = (M + CR - 1) / CR;
    {
      double2 v[D][LPT];
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (d < nch) load_chunk(d * CR, v[d]);
      for (int c0 = 0; c0 < nch; c0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int ch = c0 + d;
          if (ch >= nch) break;
          const int b = ch & 1;
          // buffer b was last read for chunk ch - 2, before chunk ch - 1's barrier
#pragma unroll
          for (int q = 0; q < LPT; ++q) {
            const int e = tid + NT * q;
            Ch[b][e % CR][e / CR] = v[d][q];
          }
          if (ch + D < nch) load_chunk((ch + D) * CR, v[d]);
          __syncthreads();
#pragma unroll 4
          for (int rr = wave; rr < CR; rr += NW) {
            double2 x[TB], y[TB];
#pragma unroll
            for (int i = 0; i < TB; ++i) x[i] = Ch[b][rr][bi * TB + i];
#pragma unroll
            for (int j = 0; j < TB; ++j) y[j] = Ch[b][rr][bj * TB + j];
#pragma unroll
            for (int i = 0; i < TB; ++i)
#pragma unroll
              for (int j = 0; j < TB; ++j) acc[i][j] = cfmac(x[i], y[j], acc[i][j]);
          }
        }
      }
    }
    for (int w = 0; w < NW; ++w) {  // the waves' sums into Gb[0], in wave order
      __syncthreads();
      if (wave == w) {
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) {
            const int gi = bi * TB + i, gj = bj * TB + j;
            Gb[0][gi][gj] = (w == 0) ? acc[i][j] : cadd(Gb[0][gi][gj], acc[i][j]);
          }
      }
    }
  }
  __syncthreads();
  if (clk) phase_clock[1] = wall_clock64();

  // 2. inner Jacobi (with many column blocks a single inner sweep per step is enough:
  //    the next steps revisit every column; with few blocks up to maxin_few sweeps)
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-53;
  const double ztol = fro2 * 0x1p-88;
  //    Within a sweep, the pairs inside each block are rotated at its first step; the
  //    later steps rotate only the pairs across the two blocks.
  const bool many = nbp >= 16;
  int cur;
  if constexpr (W2 == 32) {
    __shared__ StagedRot<W2> K;
    cur = inner_jacobi_pairs<W2, NT>(Gb, Rb, L, K, cols, many ? maxin : maxin_few, tol, ztol, many && step > 0);
  } else if constexpr (W2 == 16) {
    __shared__ StagedRot<W2> K;
    cur = inner_jacobi_staged<W2, NT>(Gb, Rb, L, K, cols, many ? maxin : maxin_few, tol, ztol, many && step > 0);
  } else {
    cur = inner_jacobi_block<W2, NT>(Gb, Rb, L, cols, many ? maxin : maxin_few, tol, ztol, many && step > 0);
  }
  const int res_rot = L.any_rot;
  if (clk) phase_clock[2] = wall_clock64();

  // 3. A_P <- A_P R and V_P <- V_P R over the JR + N rows (W's, then V's; W's alone
  //    when V is not accumulated)
  if constexpr (W2 == 16) {
    if (res_rot) {
      rot_update(rot_set(T.JW, M, nullptr, 0), cols, Rb[cur]);
      if (tid == 0) flags[sweep % 3] = 1;
    }
    if (T.jvec) {  // V's update left to the next step's blocks (or the flush)
      const int g = sweep * (nbp - 1) + step;
      const long e = vp_entry(N, g, pi);
      if (tid < 256) T.VPR[e * 256 + tid] = Rb[cur][tid / 16][tid % 16];
      if (tid < 16) T.VPC[e * 17 + tid] = cols[tid];
      if (tid == 0) T.VPC[e * 17 + 16] = res_rot ? g + 1 : 0;
    }
  } else if (res_rot) {
    const int total = M + (T.jvec ? N : 0);
    {
      const double2(*R)[W2 + 1] = Rb[cur];
      for (int r0 = 0; r0 < total; r0 += NT * RPT) {
        double2 x[RPT][W2];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int rr = r0 + tid + NT * k;
          const bool inA = rr < M;
          const double2* X = inA ? T.JW : T.JV;
          const int rows = inA ? M : N;
          const int r = inA ? rr : rr - M;
#pragma unroll
          for (int l = 0; l < W2; ++l)
            x[k][l] = (rr < total && cols[l] >= 0) ? X[(long)cols[l] * rows + r] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int rr = r0 + tid + NT * k;
          if (rr >= total) continue;
          const bool inA = rr < M;
          double2* X = inA ? T.JW : T.JV;
          const int rows = inA ? M : N;
          const int r = inA ? rr : rr - M;
#pragma unroll 4
          for (int pc = 0; pc < W2; ++pc) {
            double2 y = cmk(0.0, 0.0);
#pragma unroll
            for (int l = 0; l < W2; ++l) y = cfma(x[k][l], R[l][pc], y);
            if (cols[pc] >= 0) X[(long)cols[pc] * rows + r] = y;
          }
        }
      }
    }
    if (tid == 0) flags[sweep % 3] = 1;
  }
  if (tid < W2 && cols[tid] >= 0) T.sig2[cols[tid]] = Gb[cur][tid][tid].x;
  if (clk) {
    __threadfence();
    phase_clock[3] = wall_clock64();
    phase_clock[4] = res_rot;
  }
}

// ------------------------------------------------------------------ split Jacobi step
// The step of k_jacobi_step<8> as two launches of 256-thread blocks, two a column-block
// pair (row halves h = 0, 1), for launches that serve few updates: twice the blocks
// of half the size.
//   k_jacobi_gram: the half's partial Gram of the pair's columns of W over its rows
//     (MFMA as in the fused kernel; Re part and P = Xr^T Xi part) into JG;
//   k_jacobi_rot: both halves' partials added (h = 0 first), so that both blocks of a
//     pair form the same G, the same inner Jacobi and the same R; block h = 0 updates
//     the first half of the 16-row tiles of W and V (rot_tiles), h = 1 the rest (rot_rows).
// The launch boundary orders every Gram read of a step before its updates.
namespace {
constexpr int kSplitNT = 256;

// the pair's columns (blockIdx.x = pair + P * half); false: nothing to do
__device__ __forceinline__ bool split_pair(const Task2& T, int step, int P, int sweep, int (&cols)[16], int& pi,
                                           int& h, int& nbp) {
  constexpr int BW = 8;
  const int N = T.N;
  const int nb = (N + BW - 1) / BW;
  nbp = nb + (nb & 1);
  pi = blockIdx.x % P;
  h = blockIdx.x / P;
  if (step >= nbp - 1 || pi >= nbp / 2) return false;
  if (sweep > 0 && T.flags[(sweep + 2) % 3] == 0) return false;
  const int I = rr_player(pi, step, nbp), J = rr_player(nbp - 1 - pi, step, nbp);
  const int tid = threadIdx.x;
  if (tid < 16) {
    const int blk = tid < BW ? I : J;
    const int c = blk * BW + (tid % BW);
    cols[tid] = (blk < nb && c < N) ? T.perm[c] : -1;
  }
  __syncthreads();
  return true;
}
}  // namespace

__global__ __launch_bounds__(256) void k_jacobi_gram(Task2* tasks, const Ent* ents, int step, int P) {
  constexpr int W2 = 16, NT = kSplitNT, NW = NT / 64, KB = 16;
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int sweep = ents[blockIdx.y].sweep;
  const int tid = threadIdx.x;
  // slot (sweep+1)%3 is neither read nor written during this sweep: clear it for the
  // next one (also for converged tasks, whose later sweeps must read 0)
  if (step == 0 && blockIdx.x == 0 && tid == 0) T.flags[(sweep + 1) % 3] = 0;
  __shared__ int cols[W2];
  __shared__ double Gw[NW][2][W2][W2 + 1];
  int pi, h, nbp;
  if (!split_pair(T, step, P, sweep, cols, pi, h, nbp)) return;
  const int M = T.JR;
  const int Mh = (M + 1) / 2;
  const int r_lo = h * Mh, r_hi = min(M, r_lo + Mh);
  const double2* __restrict__ A = T.JW;
  const int wave = tid >> 6, lane = tid & 63;
  mfma_d4 gr = {0.0, 0.0, 0.0, 0.0}, gp = {0.0, 0.0, 0.0, 0.0};
  const int c = cols[lane & 15];
  const int roff = lane >> 4;
  const int nks = (r_hi - r_lo + 3) / 4;
  for (int ks0 = wave; ks0 < nks; ks0 += NW * KB) {
    double2 x[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      const int r = r_lo + (ks0 + NW * t) * 4 + roff;
      x[t] = (c >= 0 && r < r_hi) ? A[(long)c * M + r] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      gr = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].x, x[t].x, gr, 0, 0, 0);
      gr = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].y, x[t].y, gr, 0, 0, 0);
      gp = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t].x, x[t].y, gp, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Gw[wave][0][roff + 4 * r][lane & 15] = gr[r];
    Gw[wave][1][roff + 4 * r][lane & 15] = gp[r];
  }
  __syncthreads();
  double* out = T.JG + ((long)pi * 2 + h) * 2 * W2 * W2;
  for (int e = tid; e < W2 * W2; e += NT) {  // the waves' sums in wave order
    const int i = e / W2, j = e % W2;
    double sr = 0.0, sp = 0.0;
    for (int w = 0; w < NW; ++w) {
      sr += Gw[w][0][i][j];
      sp += Gw[w][1][i][j];
    }
    out[e] = sr;
    out[W2 * W2 + e] = sp;
  }
}

__global__ __launch_bounds__(256) void k_jacobi_rot(Task2* tasks, const Ent* ents, int step, int P, double tol_mult,
                                                    int maxin, int maxin_few) {
  constexpr int W2 = 16, NT = kSplitNT;
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int sweep = ents[blockIdx.y].sweep;
  const int tid = threadIdx.x;
  __shared__ int cols[W2];
  __shared__ double2 Gb[2][W2][W2 + 1];
  __shared__ double2 Rb[2][W2][W2 + 1];
  __shared__ InnerLds<W2> L;
  const double fro2 = *T.fro2;
  int pi, h, nbp;
  if (!split_pair(T, step, P, sweep, cols, pi, h, nbp)) return;
  const int N = T.N, M = T.JR;
  {  // G from the two halves' partials (h = 0 first)
    const double* g = T.JG + (long)pi * 2 * 2 * W2 * W2;
    constexpr int H1 = 2 * W2 * W2, PP = W2 * W2;
    for (int e = tid; e < W2 * W2; e += NT) {
      const int i = e / W2, j = e % W2, et = j * W2 + i;
      const double sr = g[e] + g[H1 + e];
      const double pij = g[PP + e] + g[H1 + PP + e];
      const double pji = g[PP + et] + g[H1 + PP + et];
      Gb[0][i][j] = cmk(sr, pij - pji);
    }
  }
  __syncthreads();
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-53;
  const double ztol = fro2 * 0x1p-88;
  const bool many = nbp >= 16;
  __shared__ StagedRot<W2> K;
  const int cur = inner_jacobi_staged<W2, NT>(Gb, Rb, L, K, cols, many ? maxin : maxin_few, tol, ztol, many && step > 0);
  if (L.any_rot) {  // h = 0: the matrix-core part of W's and V's update, h = 1: the vector part
    const RotSet S = rot_set(T.JW, M, T.jvec ? T.JV : nullptr, T.jvec ? N : 0);
    if (h == 0)
      rot_tiles(S, tid >> 6, NT / 64, cols, rot_operand(Rb[cur], tid & 63), tid & 63);
    else
      rot_rows(S, tid, NT, cols, Rb[cur]);
    if (tid == 0) T.flags[sweep % 3] = 1;
  }
  if (h == 0 && tid < W2 && cols[tid] >= 0) T.sig2[cols[tid]] = Gb[cur][tid][tid].x;
}

// ------------------------------------------------------------------ ordering
// In-place bitonic sort of P (a power of two) LDS (key, index) pairs, largest key
// first, equal keys by ascending index; the whole block takes part.
__device__ void bitonic_desc(double* key, int* idx, int P) {
  const int tid = threadIdx.x, nt = blockDim.x;
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
}

// Column order of a sweep (de Rijk's pivoting for one-sided Jacobi): the N columns
// of W sorted by their squared norms at the end of the previous sweep (the Gram
// diagonals every step leaves in sig2), largest first.  The step kernels pair the
// blocks of this order; sweep 0 keeps the identity order set by k_prep2.
__global__ __launch_bounds__(1024) void k_jacobi_order(Task2* tasks, const Ent* ents) {
  Task2& T = tasks[ents[blockIdx.x].slot];
  if (ents[blockIdx.x].sweep == 0) return;
  const int N = T.N;
  int P = 1;
  while (P < N) P <<= 1;
  __shared__ double key[kMaxSort];
  __shared__ int idx[kMaxSort];
  for (int j = threadIdx.x; j < P; j += blockDim.x) {
    key[j] = j < N ? fmax(T.sig2[j], 0.0) : -1.0;
    idx[j] = j;
  }
  __syncthreads();
  bitonic_desc(key, idx, P);
  for (int j = threadIdx.x; j < N; j += blockDim.x) T.perm[j] = idx[j];
}

// Column order of a QR-preconditioned task: theta_w's columns by descending norm
// (sig2 holds their squared norms), into qperm.
__global__ __launch_bounds__(1024) void k_qr_order(Task2* tasks, const Ent* ents) {
  Task2& T = tasks[ents[blockIdx.x].slot];
  if (!T.qr) return;
  const int N = T.N;
  int P = 1;
  while (P < N) P <<= 1;
  __shared__ double key[kMaxSort];
  __shared__ int idx[kMaxSort];
  for (int j = threadIdx.x; j < P; j += blockDim.x) {
    key[j] = j < N ? fmax(T.sig2[j], 0.0) : -1.0;
    idx[j] = j;
  }
  __syncthreads();
  bitonic_desc(key, idx, P);
  for (int j = threadIdx.x; j < N; j += blockDim.x) T.qperm[j] = idx[j];
}

// ------------------------------------------------------------------ truncation
// Sort sigma^2 descending (bitonic, ties by column index), suffix sums for the
// discarded weight, the kept count k = min(chi, k_eps, rank, min(M, N)), the new
// Schmidt values sigma_j / nu and the column order for the split.
__global__ __launch_bounds__(1024) void k_truncate(Task2* tasks, const Ent* ents, double floor_rel) {
  Task2& T = tasks[ents[blockIdx.x].slot];
  const int chi = T.chi;
  const double eps = T.eps;
  const int N = T.N, M = T.JM;
  int P = 1;
  while (P < N) P <<= 1;
  __shared__ double key[kMaxSort];
  __shared__ int idx[kMaxSort];
  __shared__ double sc[kMaxSort];
  __shared__ int s_rank, s_keps;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < P; j += nt) {
    key[j] = j < N ? fmax(T.sig2[j], 0.0) : -1.0;
    idx[j] = j;
  }
  if (tid == 0) { s_rank = 0; s_keps = N; }
  __syncthreads();
  bitonic_desc(key, idx, P);
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
  // Where Z is formed from W's columns (wide theta, QR), a column the Jacobi treated
  // as zero (|w|^2 <= 2^-88 ||theta_w||^2, never rotated) has no meaningful direction:
  // it is dropped whatever the rank floor keeps (with a factor 4 of margin).
  const double zfloor = (T.tr || T.qr) ? *T.fro2 * 0x1p-86 : -1.0;
  int myrank = 0;
  for (int j = tid; j < N; j += nt) {
    if (sqrt(key[j]) > floor_rel * s0 && key[j] > zfloor) ++myrank;
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
  // kept weight from the suffix sums (a fixed order of additions, so the result does
  // not depend on how the block's waves are scheduled), as the dd truncation does
  const double nu = sqrt(W - (k < N ? sc[k] : 0.0));
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
// B_{s+1}'[nu][j][gamma] = conj(Z[(j c + gamma), nu-th kept column])  (rows of Z_k^H)
__global__ __launch_bounds__(256) void k_split_right(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.z].slot];
  const int k = *T.dim_out, Nt = T.Nt, c = T.c;
  const int nu = blockIdx.y;
  if (nu >= k) return;
  const int col = T.perm[nu];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < Nt; e += gridDim.x * 256) {
    const int j = e / c, ga = e - j * c;
    T.Br[(long)(2 * nu + j) * T.ldr + ga] = cconj(T.Z[(long)col * Nt + e]);
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
  __device__ double2 b(int kk, int col) const {
    return t->Z[(long)t->perm[col] * t->Nt + kk];
  }
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

__global__ __launch_bounds__(256) void k_split_left(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int k = *t->dim_out;
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->M || tn >= k) return;
  SplitLeftOp op{t, k, 1.0 / t->stats[6]};
  cgemm_tile(op, t->M, k, t->Nt, tm, tn);
}

// Wide theta: the kept columns of W = theta_w^H V are sigma_j times the right singular
// vectors of theta_w; scale them to unit norm in place (they are orthogonal to the
// Jacobi tolerance, which is what the split needs).
__global__ __launch_bounds__(256) void k_znorm(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.z].slot];
  const int k = *T.dim_out, nu = blockIdx.y;
  if (nu >= k) return;
  const int col = T.perm[nu];
  const double s = 1.0 / sqrt(T.sig2[col]);
  for (int r = blockIdx.x * 256 + threadIdx.x; r < T.JM; r += gridDim.x * 256) {
    double2* p = T.Z + (long)col * T.JM + r;
    *p = cscale(*p, s);
  }
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
// ------------------------------------------------------------------ state set-up
// The product state |0...0> on zeroed memory: write 1.0 at each listed address
// (B_s[0][0][0] and the first Schmidt value of every bond slot) and 1 into each
// bond-dimension entry.
__global__ __launch_bounds__(256) void k_set_product(double* const* ones, long n_ones, int* dims, long n_dims) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n_ones) *ones[i] = 1.0;
  if (i < n_dims) dims[i] = 1;
}

#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_prep2(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st) {
  long nn = (long)maxN * maxN;
  int gx = (int)((nn + 255) / 256);
  if (gx > 4096) gx = 4096;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_prep2, dim3(gx, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_theta2(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_theta2, dim3((maxM + 63) / 64, (maxN + 63) / 64, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_jacobi_step(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int bw, int step,
                              double tol_mult, int maxin, int maxin_few, int defer, hipStream_t st,
                              long long* phase_clock) {
  const int nb = (maxN + bw - 1) / bw;
  if (defer && bw != 8) return hipErrorInvalidValue;
  const dim3 grid((nb + (nb & 1)) / 2 * (defer ? 2 : 1), nent);
  switch (bw) {
    case 4: hipLaunchKernelGGL(k_jacobi_step<4>, grid, dim3(512), 0, st, d_tasks, d_ents, step, tol_mult, maxin,
                                   maxin_few, 0, phase_clock); break;
    case 8: hipLaunchKernelGGL(k_jacobi_step<8>, grid, dim3(512), 0, st, d_tasks, d_ents, step, tol_mult, maxin,
                                   maxin_few, defer, phase_clock); break;
    case 16: hipLaunchKernelGGL(k_jacobi_step<16>, grid, dim3(512), 0, st, d_tasks, d_ents, step, tol_mult, maxin,
                                   maxin_few, 0, phase_clock); break;
    default: return hipErrorInvalidValue;
  }
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

// V's rotations left by the last step of each listed task's sweep
__global__ __launch_bounds__(512) void k_jacobi_vflush(Task2* tasks, const Ent* ents) {
  __shared__ int cols[16];
  __shared__ double2 R[16][17];
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int nb = (T.N + 7) / 8, nbp = nb + (nb & 1);
  const int pv = blockIdx.x;
  if (!T.jvec || pv >= nbp / 2) return;
  apply_deferred_v(T, pv, (ents[blockIdx.y].sweep + 1) * (nbp - 1), R, cols);
}

hipError_t launch_jacobi_vflush(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st) {
  const int nb = (maxN + 7) / 8;
  hipLaunchKernelGGL(k_jacobi_vflush, dim3((nb + (nb & 1)) / 2, nent), dim3(512), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_jacobi_split(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int step, double tol_mult,
                               int maxin, int maxin_few, hipStream_t st) {
  const int nb = (maxN + 7) / 8;
  const int P = (nb + (nb & 1)) / 2;
  const dim3 grid(2 * P, nent);
  hipLaunchKernelGGL(k_jacobi_gram, grid, dim3(kSplitNT), 0, st, d_tasks, d_ents, step, P);
  MPS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_jacobi_rot, grid, dim3(kSplitNT), 0, st, d_tasks, d_ents, step, P, tol_mult, maxin,
                     maxin_few);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_qr_order(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st) {
  hipLaunchKernelGGL(k_qr_order, dim3(nent), dim3(1024), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_jacobi_order(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_order, dim3(nent), dim3(1024), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_fro(Task2* d_tasks, const Ent* d_ents, int nent, long maxMN, hipStream_t st) {
  const int nch = (int)((maxMN + kFroChunk - 1) / kFroChunk);
  hipLaunchKernelGGL(k_fro_part, dim3(nch, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_fro_sum, dim3(nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_truncate(Task2* d_tasks, const Ent* d_ents, int nent, double floor_rel, hipStream_t st) {
  hipLaunchKernelGGL(k_truncate, dim3(nent), dim3(1024), 0, st, d_tasks, d_ents, floor_rel);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_split(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, int maxK, hipStream_t st,
                        bool right) {
  if (right) {
    hipLaunchKernelGGL(k_split_right, dim3((maxN + 255) / 256, maxK, nent), dim3(256), 0, st, d_tasks, d_ents);
    MPS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_split_left, dim3((maxM + 63) / 64, (maxK + 63) / 64, nent), dim3(256), 0, st, d_tasks,
                     d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_znorm(Task2* d_tasks, const Ent* d_ents, int nent, int maxJM, int maxK, hipStream_t st) {
  hipLaunchKernelGGL(k_znorm, dim3((maxJM + 255) / 256, maxK, nent), dim3(256), 0, st, d_tasks, d_ents);
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

hipError_t launch_set_product(double* const* ones, long n_ones, int* dims, long n_dims, hipStream_t st) {
  const long n = n_ones > n_dims ? n_ones : n_dims;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_product, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ones, n_ones, dims, n_dims);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_amplitude(const AmpArgs& args, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_amplitude, dim3(count), dim3(256), 0, st, args);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
