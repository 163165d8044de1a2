// Double-double refinement path of the two-site update (gfx950).
//
// The state lives in double-double (hi + lo planes).  Per update:
//   theta, theta_w in dd                       [k_theta2_dd: dd GEMM + U epilogue]
//   FP64 block Jacobi on round(theta_w)        [k_jacobi_step<BW> of kernels.hip] -> V0
//   V <- V (I - E/2), E = V^H V - I, twice     [k_gram_dd + k_ns_fix] (Newton-Schulz step of
//                                              the polar factor: orthogonality error squares)
//   W = theta_w V in dd                        [k_wmul_dd]  (theta_w^H V for a wide theta)
//   dd block Jacobi polish sweeps on (W, V)    [k_jacobi_step_dd]
//   sort / truncate / renormalise in dd        [k_truncate_dd]
//   B_{s+1}' = Z_k^H, B_s' = theta Z_k / nu    [k_split_*_dd]
// No step divides by a Schmidt value (same gauge as the FP64 path).
#include "dd.h"
#include "dd_kernels.h"
#include "gemm.h"
#include "ddgemm.h"

namespace mpsk {

using dd::cacc;
using dd::cdd;
using dd::ddr;

// ------------------------------------------------------------------ single-site gate
__global__ __launch_bounds__(256) void k_gate1_dd(Task1* tasks) {
  const Task1& T = tasks[blockIdx.y];
  const long nel = (long)T.a * T.b;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nel; e += (long)gridDim.x * 256) {
    const int al = (int)(e / T.b), be = (int)(e - (long)al * T.b);
    const long i0 = (long)(2 * al) * T.ld + be, i1 = i0 + T.ld;
    const cdd x0 = ldc(T.B, T.B_lo, i0), x1 = ldc(T.B, T.B_lo, i1);
    cacc y0 = cacc0(), y1 = cacc0();
    dd::cacc_fma(y0, ld_gate(T.U, T.U_lo, 0), x0);
    dd::cacc_fma(y0, ld_gate(T.U, T.U_lo, 1), x1);
    dd::cacc_fma(y1, ld_gate(T.U, T.U_lo, 2), x0);
    dd::cacc_fma(y1, ld_gate(T.U, T.U_lo, 3), x1);
    stc(T.B, T.B_lo, i0, dd::cnorm(y0));
    stc(T.B, T.B_lo, i1, dd::cnorm(y1));
  }
}

// ------------------------------------------------------------------ theta (2 sites)
// Same contraction as the FP64 k_theta2 (B-operand columns 2*gamma + j'), each
// thread's 2 x 2 block is one (alpha, gamma) with its four (i', j') entries.
struct ThetaOpDD {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = true;
  const Task2* t;
  __device__ cdd a(int row, int kk) const { return ldc(t->Bl, t->Bl_lo, (long)row * t->ldl + kk); }
  __device__ cdd b(int kk, int col) const {
    return ldc(t->Br, t->Br_lo, (long)(2 * kk + (col & 1)) * t->ldr + (col >> 1));
  }
  __device__ void epilogue(int r0, int c0, cdd (&T4)[2][2]) const {
    const int al = r0 >> 1, ga = c0 >> 1, M = t->M;
    if (al < t->a && ga < t->c) {
      const ddr wl = {t->lamL[al], t->lamL_lo[al]};
      cdd Tin[4] = {T4[0][0], T4[0][1], T4[1][0], T4[1][1]};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cacc o = cacc0();
#pragma unroll
          for (int q = 0; q < 4; ++q) dd::cacc_fma(o, ld_gate(t->U, t->U_lo, (i * 2 + j) * 4 + q), Tin[q]);
          const cdd v = dd::cnorm(o);
          const long idx = (long)(j * t->c + ga) * M + (2 * al + i);
          stc(t->thu, t->thu_lo, idx, v);
          const cdd w = dd::cscale(v, wl);
          if (t->tr)
            t->thw[(long)(2 * al + i) * t->Nt + (j * t->c + ga)] = make_double2(w.re.hi, -w.im.hi);
          else
            t->thw[idx] = make_double2(w.re.hi, w.im.hi);
        }
    }
  }
};

__global__ __launch_bounds__(256) void k_theta2_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->M || tn >= t->Nt) return;
  ThetaOpDD op{t};
  ddgemm_tile(op, t->M, t->Nt, t->b, tm, tn);
}

// ------------------------------------------------------------------ Newton-Schulz
// E = V^H V - I (dd accumulation, stored binary64: E is of the size of V's
// orthogonality error, so its binary64 rounding is far below dd precision of V).
// E is Hermitian: only the tiles on and above the diagonal are formed, an
// off-diagonal tile also writing its conjugate transpose.
struct GramOpDD {
  static constexpr bool kARowFast = false;
  static constexpr bool kBColFast = false;
  const Task2* t;
  bool mirror;
  __device__ cdd a(int row, int kk) const { return dd::cconj(ldc(t->V, t->V_lo, (long)row * t->N + kk)); }
  __device__ cdd b(int kk, int col) const { return ldc(t->V, t->V_lo, (long)col * t->N + kk); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
    const int N = t->N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r >= N || c >= N) continue;
        cdd e = v[i][j];
        if (r == c) e.re = dd::add_d(e.re, -1.0);
        t->aux1[(long)c * N + r] = make_double2(e.re.hi, e.im.hi);  // column-major
        if (mirror) t->aux1[(long)r * N + c] = make_double2(e.re.hi, -e.im.hi);
      }
  }
};

__global__ __launch_bounds__(256) void k_gram_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->N || tn >= t->N || tm > tn) return;
  GramOpDD op{t, tm != tn};
  ddgemm_tile(op, t->N, t->N, t->N, tm, tn);
}

// C = V_hi E (binary64), into aux2
struct NsOp {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  __device__ double2 a(int row, int kk) const { return t->V[(long)kk * t->N + row]; }
  __device__ double2 b(int kk, int col) const { return t->aux1[(long)col * t->N + kk]; }
  __device__ void epilogue(int r0, int c0, double2 (&acc)[4][4]) const {
    const int N = t->N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r < N && c < N) t->aux2[(long)c * N + r] = acc[i][j];
      }
  }
};

__global__ __launch_bounds__(256) void k_ns_mul(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 64, tn = blockIdx.y * 64;
  if (tm >= t->N || tn >= t->N) return;
  NsOp op{t};
  cgemm_tile(op, t->N, t->N, t->N, tm, tn);
}

// V <- V - C / 2 (dd minus binary64)
__global__ __launch_bounds__(256) void k_ns_fix(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const long nn = (long)T.N * T.N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
    cdd v = ldc(T.V, T.V_lo, e);
    const double2 c = T.aux2[e];
    v.re = dd::add_d(v.re, -0.5 * c.x);
    v.im = dd::add_d(v.im, -0.5 * c.y);
    stc(T.V, T.V_lo, e, v);
  }
}

// promote V (binary64 from the FP64 Jacobi) to dd, clear the rotation flags
__global__ __launch_bounds__(256) void k_promote(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const long nn = (long)T.N * T.N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256)
    T.V_lo[e] = make_double2(0.0, 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) T.flags[0] = T.flags[1] = T.flags[2] = 0;
}

// ------------------------------------------------------------------ W = theta_w V
struct WOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  __device__ cdd a(int row, int kk) const {
    if (t->tr) {  // theta_w^H: row = theta column, kk = theta row
      const cdd x = ldc(t->thu, t->thu_lo, (long)row * t->M + kk);
      const ddr w = {t->lamL[kk >> 1], t->lamL_lo[kk >> 1]};
      return dd::cconj(dd::cscale(x, w));
    }
    const cdd x = ldc(t->thu, t->thu_lo, (long)kk * t->M + row);
    const ddr w = {t->lamL[row >> 1], t->lamL_lo[row >> 1]};
    return dd::cscale(x, w);
  }
  __device__ cdd b(int kk, int col) const { return ldc(t->V, t->V_lo, (long)col * t->N + kk); }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + i, c = c0 + j;
        if (r < t->JM && c < t->N) stc(t->thw, t->thw_lo, (long)c * t->JM + r, v[i][j]);
      }
  }
};

__global__ __launch_bounds__(256) void k_wmul_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->JM || tn >= t->N) return;
  WOpDD op{t};
  ddgemm_tile(op, t->JM, t->N, t->N, tm, tn);
}

// ------------------------------------------------------------------ dd Jacobi step
// The block one-sided Jacobi step of kernels.hip in double-double: dd Gram of the
// pair, dd two-sided Jacobi on it, dd update of W and V.  The rotation angle is
// formed in binary64 from the dd Gram entries (an angle error of 2^-53 relative only
// leaves an off-diagonal residual 2^-53 times the one being removed, which the
// polish then removes), while c, s and the phase e are completed in dd so that
// every applied rotation is unitary to dd precision.
__device__ __forceinline__ int rrp(int i, int r, int np) { return i == 0 ? 0 : 1 + (i - 1 + r) % (np - 1); }

__device__ __forceinline__ double rcp_nr_dd(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr_dd(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// coefficients of index p (ap, bp) and q (aq, bq): (X J)[:, x] = a_x X_x + b_x X_partner
__device__ __forceinline__ bool dd_pair_rot(ddr al, ddr be, cdd g, double tol, double ztol, cdd& ap, cdd& bp,
                                            cdd& aq, cdd& bq) {
  const double gr = g.re.hi, gi = g.im.hi;
  const double g2 = gr * gr + gi * gi;
  if (!(al.hi > ztol && be.hi > ztol && g2 > tol * tol * al.hi * be.hi)) return false;
  const double ig = rsq_nr_dd(g2);
  const double zeta = 0.5 * dd::sub(be, al).hi * ig;
  double t = rcp_nr_dd(fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
  t = zeta < 0.0 ? -t : t;
  // c = 1 / sqrt(1 + t^2), s = t c, in dd
  const ddr one_t2 = dd::add_d(dd::two_prod(t, t), 1.0);
  const ddr c = dd::div(dd::from(1.0), dd::sqrt(one_t2));
  const ddr sn = dd::mul_d(c, t);
  // unit phase e = conj(g) / |g|: binary64 estimate, normalised in dd
  const double er = gr * ig, ei = -gi * ig;
  const ddr n2 = dd::add(dd::two_prod(er, er), dd::two_prod(ei, ei));
  const ddr inv = dd::div(dd::from(1.0), dd::sqrt(n2));
  const cdd e = {dd::mul_d(inv, er), dd::mul_d(inv, ei)};
  ap = {c, {0.0, 0.0}};
  bp = dd::cscale(e, dd::neg(sn));
  aq = dd::cscale(e, c);
  bq = {sn, {0.0, 0.0}};
  return true;
}

__global__ __launch_bounds__(256) void k_jacobi_step_dd(Task2* tasks, const Ent* ents, int step, double tol_mult,
                                                         int maxin) {
  constexpr int BW = 8, W2 = 16, TB = 2, LPT = 64 * W2 / 256;
  const Task2& T = tasks[ents[blockIdx.y].slot];
  const int sweep = ents[blockIdx.y].sweep;
  const int N = T.N, M = T.JM;
  const int nb = (N + BW - 1) / BW;
  const int nbp = nb + (nb & 1);
  const int pi = blockIdx.x;
  if (step >= nbp - 1 || pi >= nbp / 2) return;
  int* flags = T.flags;
  const int tid = threadIdx.x;
  if (step == 0 && pi == 0 && tid == 0) flags[(sweep + 1) % 3] = 0;
  if (sweep > 0 && flags[(sweep + 2) % 3] == 0) return;

  __shared__ int cols[W2];
  __shared__ double2 Chh[64][W2 + 1], Chl[64][W2 + 1];
  __shared__ cdd Gb[2][W2][W2 + 1];
  __shared__ cdd Rb[2][W2][W2 + 1];
  __shared__ cdd ca[W2], cb[W2];
  __shared__ int cpart[W2], crot[W2];
  __shared__ int rnd_rot[2];
  __shared__ int swf[3];
  __shared__ int any_rot;

  const int I = rrp(pi, step, nbp), J = rrp(nbp - 1 - pi, step, nbp);
  if (tid < W2) {
    const int blk = tid < BW ? I : J;
    const int c = blk * BW + (tid % BW);
    cols[tid] = (blk < nb && c < N) ? c : -1;
  }
  if (tid < 3) swf[tid] = 0;
  if (tid < 2) rnd_rot[tid] = 0;
  if (tid == 0) any_rot = 0;
  __syncthreads();

  // 1. dd Gram; the next chunk's loads are issued before the current chunk is reduced
  const int wave = tid >> 6, lane = tid & 63;
  const int bi = lane >> 3, bj = lane & 7;
  cacc acc[TB][TB];
#pragma unroll
  for (int i = 0; i < TB; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = cacc0();
  auto load = [&](int r0, double2 (&vh)[LPT], double2 (&vl)[LPT]) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + 256 * q;
      const int rr = e & 63, l = e >> 6;
      const int c = cols[l], r = r0 + rr;
      const bool ok = c >= 0 && r < M;
      vh[q] = ok ? T.thw[(long)c * M + r] : make_double2(0.0, 0.0);
      vl[q] = ok ? T.thw_lo[(long)c * M + r] : make_double2(0.0, 0.0);
    }
  };
  {
    double2 vh[LPT], vl[LPT];
    load(0, vh, vl);
    for (int r0 = 0; r0 < M; r0 += 64) {
      __syncthreads();  // the previous chunk has been reduced
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int e = tid + 256 * q;
        Chh[e & 63][e >> 6] = vh[q];
        Chl[e & 63][e >> 6] = vl[q];
      }
      if (r0 + 64 < M) load(r0 + 64, vh, vl);
      __syncthreads();
      for (int rr = wave; rr < 64; rr += 4) {
        cdd x[TB], y[TB];
#pragma unroll
        for (int i = 0; i < TB; ++i) {
          const double2 h = Chh[rr][bi * TB + i], l = Chl[rr][bi * TB + i];
          x[i] = {{h.x, l.x}, {h.y, l.y}};
        }
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const double2 h = Chh[rr][bj * TB + j], l = Chl[rr][bj * TB + j];
          y[j] = {{h.x, l.x}, {h.y, l.y}};
        }
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) dd::cacc_fmac(acc[i][j], x[i], y[j]);
      }
    }
  }
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const int gi = bi * TB + i, gj = bj * TB + j;
          const cdd v = dd::cnorm(acc[i][j]);
          Gb[0][gi][gj] = (w == 0) ? v : dd::cadd(Gb[0][gi][gj], v);
        }
    }
  }
  for (int e = tid; e < W2 * W2; e += 256) {
    const int i = e / W2, j = e % W2;
    Rb[0][i][j] = {{i == j ? 1.0 : 0.0, 0.0}, {0.0, 0.0}};
  }
  const double tol = tol_mult * (double)(M > 16 ? M : 16) * 0x1p-101;
  const double ztol = *T.fro2 * 0x1p-192;  // columns below 2^-96 ||theta|| are rounding noise
  __syncthreads();

  // 2. two-sided Jacobi on G in dd: one thread per pair forms the rotation, then every
  //    thread forms its element of J^H G J and R J (double-buffered)
  // the polish diagonalises each pair's nearly diagonal Gram fully (rounds without
  // a rotation cost only the coefficient check)
  const int inner = maxin > 12 ? maxin : 12;
  int cur = 0;
  for (int isw = 0; isw < inner; ++isw) {
    if (tid == 0) swf[(isw + 1) % 3] = 0;
    for (int rnd = 0; rnd < W2 - 1; ++rnd) {
      if (tid < W2 / 2) {
        const int pa = rrp(tid, rnd, W2), pb = rrp(W2 - 1 - tid, rnd, W2);
        const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
        cdd ap, bp, aq, bq;
        const bool rot = cols[p] >= 0 && cols[q] >= 0 &&
                         dd_pair_rot(Gb[cur][p][p].re, Gb[cur][q][q].re, Gb[cur][p][q], tol, ztol, ap, bp, aq, bq);
        if (!rot) {
          ap = aq = {{1.0, 0.0}, {0.0, 0.0}};
          bp = bq = czero();
        } else {
          swf[isw % 3] = 1;
          rnd_rot[rnd & 1] = 1;
        }
        ca[p] = ap; cb[p] = bp; ca[q] = aq; cb[q] = bq;
        cpart[p] = q; cpart[q] = p;
        crot[p] = rot; crot[q] = rot;
      }
      __syncthreads();
      if (tid == 0) rnd_rot[(rnd + 1) & 1] = 0;
      if (!rnd_rot[rnd & 1]) {
        __syncthreads();
        continue;
      }
      {
        const int i = tid / W2, j = tid % W2;
        const int pi_ = cpart[i], pj = cpart[j];
        const cdd ai = ca[i], bi_ = cb[i], aj = ca[j], bj_ = cb[j];
        const cdd (*G)[W2 + 1] = Gb[cur];
        const cdd colj = dd::cadd(dd::cmul(aj, G[i][j]), dd::cmul(bj_, G[i][pj]));
        const cdd colpj = dd::cadd(dd::cmul(aj, G[pi_][j]), dd::cmul(bj_, G[pi_][pj]));
        cdd v = dd::cadd(dd::cmul(dd::cconj(ai), colj), dd::cmul(dd::cconj(bi_), colpj));
        if (crot[i] && j == pi_) v = czero();
        if (i == j) v.im = {0.0, 0.0};
        const cdd rn = dd::cadd(dd::cmul(aj, Rb[cur][i][j]), dd::cmul(bj_, Rb[cur][i][pj]));
        Gb[cur ^ 1][i][j] = v;
        Rb[cur ^ 1][i][j] = rn;
      }
      cur ^= 1;
      __syncthreads();
    }
    if (!swf[isw % 3]) break;
    if (tid == 0) any_rot = 1;
  }
  __syncthreads();

  // 3. dd update of the pair's columns of W and V (M + N rows, a row per thread at a
  //    time, all its loads issued before the products)
  if (any_rot) {
    const int total = M + N;
    for (int rr = tid; rr < total; rr += 256) {
      const bool inA = rr < M;
      double2* Xh = inA ? T.thw : T.V;
      double2* Xl = inA ? T.thw_lo : T.V_lo;
      const int rows = inA ? M : N;
      const int r = inA ? rr : rr - M;
      cdd x[W2];
#pragma unroll
      for (int l = 0; l < W2; ++l) x[l] = cols[l] >= 0 ? ldc(Xh, Xl, (long)cols[l] * rows + r) : czero();
#pragma unroll 1
      for (int pc = 0; pc < W2; ++pc) {
        cacc y = cacc0();
#pragma unroll 4
        for (int l = 0; l < W2; ++l) dd::cacc_fma(y, x[l], Rb[cur][l][pc]);
        if (cols[pc] >= 0) stc(Xh, Xl, (long)cols[pc] * rows + r, dd::cnorm(y));
      }
    }
    if (tid == 0) flags[sweep % 3] = 1;
  }
  if (tid < W2 && cols[tid] >= 0) {
    T.sig2[cols[tid]] = Gb[cur][tid][tid].re.hi;
    T.sig2_lo[cols[tid]] = Gb[cur][tid][tid].re.lo;
  }
}

// ------------------------------------------------------------------ truncation (dd)
__device__ __forceinline__ bool dd_before(ddr a, int ia, ddr b, int ib) {
  return dd::lt(b, a) || (a.hi == b.hi && a.lo == b.lo && ia < ib);
}

__global__ __launch_bounds__(1024) void k_truncate_dd(Task2* tasks, const Ent* ents, double floor_rel) {
  Task2& T = tasks[ents[blockIdx.x].slot];
  const int chi = T.chi;
  const double eps = T.eps;
  const int N = T.N, M = T.JM;
  int P = 1;
  while (P < N) P <<= 1;
  __shared__ ddr key[kMaxSort];
  __shared__ int idx[kMaxSort];
  __shared__ ddr sc[kMaxSort];
  __shared__ int s_rank, s_keps;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < P; j += nt) {
    if (j < N) {
      ddr v = {T.sig2[j], T.sig2_lo[j]};
      if (v.hi < 0) v = {0.0, 0.0};
      key[j] = v;
    } else {
      key[j] = {-1.0, 0.0};
    }
    idx[j] = j;
  }
  if (tid == 0) { s_rank = 0; s_keps = N; }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += nt) {
        const int l = i ^ stride;
        if (l > i) {
          const bool before = dd_before(key[i], idx[i], key[l], idx[l]);
          const bool dir = (i & size) == 0;
          if (dir != before) {
            const ddr tk = key[i]; key[i] = key[l]; key[l] = tk;
            const int ti = idx[i]; idx[i] = idx[l]; idx[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < P; j += nt) sc[j] = j < N ? key[j] : ddr{0.0, 0.0};
  __syncthreads();
  for (int off = 1; off < P; off <<= 1) {
    ddr v[kMaxSort / 1024];
    int cnt = 0;
    for (int j = tid; j < P; j += nt) v[cnt++] = (j + off < P) ? sc[j + off] : ddr{0.0, 0.0};
    __syncthreads();
    cnt = 0;
    for (int j = tid; j < P; j += nt) { sc[j] = dd::add(sc[j], v[cnt]); ++cnt; }
    __syncthreads();
  }
  const ddr W = sc[0];
  const double s0 = sqrt(key[0].hi);
  const ddr epsW = dd::mul_d(W, eps);
  // as in the FP64 truncation: with Z formed from W's columns (wide theta, or a QR
  // task refined as the transposed problem), columns the dd Jacobi treated as zero
  // (|w|^2 <= 2^-192 ||theta_w||^2) are dropped
  const double zfloor = (T.tr || T.qr) ? *T.fro2 * 0x1p-190 : -1.0;
  int myrank = 0;
  for (int j = tid; j < N; j += nt) {
    if (sqrt(key[j].hi) > floor_rel * s0 && key[j].hi > zfloor) ++myrank;
    const int kk = j + 1;
    const ddr tailk = kk < N ? sc[kk] : ddr{0.0, 0.0};
    if (!dd::lt(epsW, tailk)) atomicMin(&s_keps, kk);
  }
  atomicAdd(&s_rank, myrank);
  __syncthreads();
  int k = chi;
  if (s_keps < k) k = s_keps;
  if (s_rank < k) k = s_rank;
  const int mn = M < N ? M : N;
  if (mn < k) k = mn;
  if (k < 1) k = 1;
  const ddr tail = k < N ? sc[k] : ddr{0.0, 0.0};
  const ddr nu = dd::sqrt(dd::sub(W, tail));
  for (int j = tid; j < N; j += nt) {
    T.perm[j] = idx[j];
    if (j < k) {
      const ddr l = dd::div(dd::sqrt(key[j]), nu);
      T.lamS[j] = l.hi;
      T.lamS_lo[j] = l.lo;
    }
  }
  if (tid == 0) {
    double* st = T.stats;
    st[0] = W.hi;
    st[1] = W.hi > 0 ? dd::div(tail, W).hi : 0.0;
    st[2] = (k < s_rank) ? (dd::sub(dd::sqrt(key[k - 1]), dd::sqrt(key[k]))).hi / s0 : INFINITY;
    double ed = INFINITY;
    if (eps > 0) {
      for (int kk = s_keps - 1; kk <= s_keps; ++kk) {
        if (kk < 1 || kk > N) continue;
        const ddr tk = kk < N ? sc[kk] : ddr{0.0, 0.0};
        const double d = fabs(dd::sub(tk, epsW).hi) / epsW.hi;
        ed = d < ed ? d : ed;
      }
    }
    st[3] = ed;
    st[4] = k;
    st[5] = s_rank;
    st[6] = nu.hi;
    st[7] = nu.lo;
    *T.dim_out = k;
  }
}

// ------------------------------------------------------------------ split (dd)
__global__ __launch_bounds__(256) void k_split_right_dd(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.z].slot];
  const int k = *T.dim_out, Nt = T.Nt, c = T.c;
  const int nu = blockIdx.y;
  if (nu >= k) return;
  const int col = T.perm[nu];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < Nt; e += gridDim.x * 256) {
    const int j = e / c, ga = e - j * c;
    const cdd v = dd::cconj(ldc(T.Z, T.Z_lo, (long)col * Nt + e));
    stc(T.Br, T.Br_lo, (long)(2 * nu + j) * T.ldr + ga, v);
  }
}

struct SplitLeftOpDD {
  static constexpr bool kARowFast = true;
  static constexpr bool kBColFast = false;
  const Task2* t;
  int k;
  ddr inv_nu;
  __device__ cdd a(int row, int kk) const { return ldc(t->thu, t->thu_lo, (long)kk * t->M + row); }
  __device__ cdd b(int kk, int col) const {
    return ldc(t->Z, t->Z_lo, (long)t->perm[col] * t->Nt + kk);
  }
  __device__ void epilogue(int r0, int c0, cdd (&v)[2][2]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = r0 + i, cc = c0 + j;
        if (r < t->M && cc < k) stc(t->Bl, t->Bl_lo, (long)r * t->ldl + cc, dd::cscale(v[i][j], inv_nu));
      }
  }
};

__global__ __launch_bounds__(256) void k_split_left_dd(Task2* tasks, const Ent* ents) {
  const Task2* t = &tasks[ents[blockIdx.z].slot];
  const int k = *t->dim_out;
  const int tm = blockIdx.x * 32, tn = blockIdx.y * 32;
  if (tm >= t->M || tn >= k) return;
  const ddr nu = {t->stats[6], t->stats[7]};
  SplitLeftOpDD op{t, k, dd::div(dd::from(1.0), nu)};
  ddgemm_tile(op, t->M, k, t->Nt, tm, tn);
}

// wide theta: Z = the kept columns of W scaled to unit norm, in dd
__global__ __launch_bounds__(256) void k_znorm_dd(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.z].slot];
  const int k = *T.dim_out, nu = blockIdx.y;
  if (nu >= k) return;
  const int col = T.perm[nu];
  const ddr s = dd::div(dd::from(1.0), dd::sqrt(ddr{T.sig2[col], T.sig2_lo[col]}));
  for (int r = blockIdx.x * 256 + threadIdx.x; r < T.JM; r += gridDim.x * 256) {
    const long o = (long)col * T.JM + r;
    stc(T.Z, T.Z_lo, o, dd::cscale(ldc(T.Z, T.Z_lo, o), s));
  }
}

// ------------------------------------------------------------------ amplitudes (dd)
__global__ __launch_bounds__(256) void k_amplitude_dd(const AmpArgs args, const double2* const* Blo) {
  __shared__ cdd v[1024], w[1024];
  const int tid = threadIdx.x;
  const unsigned char* bits = args.bits + (long)blockIdx.x * args.n;
  if (tid == 0) v[0] = {{1.0, 0.0}, {0.0, 0.0}};
  __syncthreads();
  for (int s = 0; s < args.n; ++s) {
    const int ml = args.dimx[s], mr = args.dimx[s + 1];
    const int b = bits[s] ? 1 : 0;
    const double2* Bh = args.B[s];
    const double2* Bl = Blo[s];
    const int ld = args.ld[s];
    for (int be = tid; be < mr; be += 256) {
      cacc acc = cacc0();
      for (int al = 0; al < ml; ++al) dd::cacc_fma(acc, v[al], ldc(Bh, Bl, (long)(2 * al + b) * ld + be));
      w[be] = dd::cnorm(acc);
    }
    __syncthreads();
    for (int be = tid; be < mr; be += 256) v[be] = w[be];
    __syncthreads();
  }
  if (tid == 0) {
    double2* o = args.out + 2 * blockIdx.x;
    o[0] = make_double2(v[0].re.hi, v[0].re.lo);
    o[1] = make_double2(v[0].im.hi, v[0].im.lo);
  }
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

bool dd_available() { return true; }

static int grid_for(long n) {
  long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_gate1_dd(Task1* d_tasks, int ntask, long maxel, hipStream_t st) {
  hipLaunchKernelGGL(k_gate1_dd, dim3(grid_for(maxel), ntask), dim3(256), 0, st, d_tasks);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_theta2_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_theta2_dd, dim3((maxM + 31) / 32, (maxN + 31) / 32, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

// Enter the dd polish: V0 (binary64) -> dd, two Newton-Schulz steps, W = theta_w V in dd.
hipError_t launch_dd_enter(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st) {
  const long nn = (long)maxN * maxN;
  hipLaunchKernelGGL(k_promote, dim3(grid_for(nn), nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  for (int it = 0; it < 2; ++it) {
    hipLaunchKernelGGL(k_gram_dd, dim3((maxN + 31) / 32, (maxN + 31) / 32, nent), dim3(256), 0, st, d_tasks, d_ents);
    hipLaunchKernelGGL(k_ns_mul, dim3((maxN + 63) / 64, (maxN + 63) / 64, nent), dim3(256), 0, st, d_tasks, d_ents);
    hipLaunchKernelGGL(k_ns_fix, dim3(grid_for(nn), nent), dim3(256), 0, st, d_tasks, d_ents);
    MPS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_wmul_dd, dim3((maxM + 31) / 32, (maxN + 31) / 32, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

// One dd polish step (inner sweeps per block pair as in the FP64 step).
hipError_t launch_jacobi_step_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int step, double tol_mult,
                                 int maxin, hipStream_t st) {
  const int nb = (maxN + 7) / 8;
  const int nbp = nb + (nb & 1);
  hipLaunchKernelGGL(k_jacobi_step_dd, dim3(nbp / 2, nent), dim3(256), 0, st, d_tasks, d_ents, step, tol_mult, maxin);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_znorm_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxJM, int maxK, hipStream_t st) {
  hipLaunchKernelGGL(k_znorm_dd, dim3((maxJM + 255) / 256, maxK, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_truncate_dd(Task2* d_tasks, const Ent* d_ents, int nent, double floor_rel, hipStream_t st) {
  hipLaunchKernelGGL(k_truncate_dd, dim3(nent), dim3(1024), 0, st, d_tasks, d_ents, floor_rel);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_split_dd(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, int maxK, hipStream_t st,
                           bool right) {
  if (right) {
    hipLaunchKernelGGL(k_split_right_dd, dim3((maxN + 255) / 256, maxK, nent), dim3(256), 0, st, d_tasks, d_ents);
    MPS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_split_left_dd, dim3((maxM + 31) / 32, (maxK + 31) / 32, nent), dim3(256), 0, st, d_tasks,
                     d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_amplitude_dd(const AmpArgs& args, const double2* const* B_lo, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_amplitude_dd, dim3(count), dim3(256), 0, st, args, B_lo);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
