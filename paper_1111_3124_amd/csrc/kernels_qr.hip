// Householder QR preconditioning of the two-site Jacobi problem (gfx950, FP64).
//
// For theta_w (M x N, M >= N) with its columns taken in descending norm order P,
// theta_w P = Q R (Householder, panels of 16 columns in compact WY form), and the
// one-sided Jacobi then runs on X = R^H (N x N): the rows of R are graded by the
// column ordering, so the Jacobi converges in fewer sweeps than on theta_w itself
// (Drmac & Veselic's preconditioner for one-sided Jacobi).  With X V_x = W_x:
//   theta_w = (Q V_x) Sigma (P U_x)^H,  U_x = W_x Sigma^-1,
// so the right singular vectors the split needs are P times the normalised kept
// columns of W_x (k_qr_z), and the left ones Q V_x (k_qr_apply in mode 1, for the
// double-double refinement of the transposed problem).
//
// Storage (in the task's workspace): the reflectors overwrite theta_w in place
// (column qperm[c] holds v_c below row c and R's row c on and above it, R[c][c] =
// beta_c on the diagonal); v_c's first entry is qvd[c] and its scale 2 / v_c^H v_c is
// qt[c]; the 16 x 16 triangular factor of panel p is qT[256 p ...].
#include "common.h"
#include "launch.h"

namespace mpsk {

namespace {

constexpr int kPanel = 16;

// Cross-lane exchanges of one wavefront on the vector ALUs (no LDS traffic): the
// value of lane l ^ 8, ^ 4, ^ 2 or ^ 1 by DPP row operations, and the two half-wave
// swaps of gfx950.  Each moves the two 32-bit halves of a double.
__device__ __forceinline__ double dbl(int lo, int hi) {
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int H>
__device__ __forceinline__ double lane_xor(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)b, hi = (int)(b >> 32);
  if constexpr (H == 8) {  // row_ror:8
    return dbl(__builtin_amdgcn_mov_dpp(lo, 0x128, 0xf, 0xf, false), __builtin_amdgcn_mov_dpp(hi, 0x128, 0xf, 0xf, false));
  } else if constexpr (H == 4) {  // row_shl:4 into lanes with bit 2 clear, row_shr:4 into the others
    int l2 = __builtin_amdgcn_update_dpp(lo, lo, 0x104, 0xf, 0x5, false);
    int h2 = __builtin_amdgcn_update_dpp(hi, hi, 0x104, 0xf, 0x5, false);
    l2 = __builtin_amdgcn_update_dpp(l2, lo, 0x114, 0xf, 0xa, false);
    h2 = __builtin_amdgcn_update_dpp(h2, hi, 0x114, 0xf, 0xa, false);
    return dbl(l2, h2);
  } else if constexpr (H == 2) {  // quad_perm [2, 3, 0, 1]
    return dbl(__builtin_amdgcn_mov_dpp(lo, 0x4e, 0xf, 0xf, false), __builtin_amdgcn_mov_dpp(hi, 0x4e, 0xf, 0xf, false));
  } else {  // quad_perm [1, 0, 3, 2]
    static_assert(H == 1, "lane_xor takes 8, 4, 2 or 1");
    return dbl(__builtin_amdgcn_mov_dpp(lo, 0xb1, 0xf, 0xf, false), __builtin_amdgcn_mov_dpp(hi, 0xb1, 0xf, 0xf, false));
  }
}
// x + y over the pair (l, l ^ H) for H = 32 or 16 (v_permlane32_swap / v_permlane16_swap
// exchange the upper half of x's lanes with the lower half of y's): lanes with bit H
// clear get their x plus the partner's x, the others their y plus the partner's y
template <int H>
__device__ __forceinline__ double swap_add(double x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const unsigned xl = (unsigned)bx, xh = (unsigned)(bx >> 32), yl = (unsigned)by, yh = (unsigned)(by >> 32);
  if constexpr (H == 32) {
    const auto rl = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    return dbl(rl[0], rh[0]) + dbl(rl[1], rh[1]);
  } else {
    static_assert(H == 16, "swap_add takes 32 or 16");
    const auto rl = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    return dbl(rl[0], rh[0]) + dbl(rl[1], rh[1]);
  }
}

// Deterministic block sum of K <= 64 doubles per thread (NW waves): a recursive-halving
// reduce-scatter inside each wave (63 lane exchanges for any K), after the exchange at
// distance 32, 16, ..., 1 lane l holds the wave's sum of value l; then the waves' sums
// in wave order; every thread gets the totals.  At each distance a lane adds its own
// value and its partner's (IEEE addition commutes, so the order within a pair does not
// matter).
template <int K, int NW>
__device__ __forceinline__ void block_sum64(double (&v)[K], double (&red)[NW][K], double (&tot)[K]) {
  static_assert(K <= 64, "block_sum64 takes at most 64 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double a[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) a[k] = k < K ? v[k] : 0.0;
  // distances 32 and 16: the lower half of the lanes keeps values [0, h), the upper [h, 2h)
#pragma unroll
  for (int i = 0; i < 32; ++i) a[i] = swap_add<32>(a[i], a[32 + i]);
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = swap_add<16>(a[i], a[16 + i]);
  auto level = [&](auto hc) {
    constexpr int h = decltype(hc)::value;
    const bool up = (lane & h) != 0;  // keep the upper half of the live values
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = up ? a[i] : a[h + i];
      const double keep = up ? a[h + i] : a[i];
      a[i] = keep + lane_xor<h>(send);
    }
  };
  level(std::integral_constant<int, 8>{});
  level(std::integral_constant<int, 4>{});
  level(std::integral_constant<int, 2>{});
  level(std::integral_constant<int, 1>{});
  if (lane < K) red[wave][lane] = a[0];
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = tot[k];
}

}  // namespace

// Squared norms of the N columns of theta_w (into sig2): one wavefront a column.
__global__ __launch_bounds__(256) void k_qr_colnorm(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  if (!T.qr) return;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= T.N) return;
  const double2* col = T.thw + (long)c * T.M;
  double s = 0.0;
  for (int r = lane; r < T.M; r += 64) s = fma(col[r].x, col[r].x, fma(col[r].y, col[r].y, s));
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) T.sig2[c] = s;
}

// One panel of 16 columns (positions p0.. of the order qperm), one 512-thread block
// per task: the panel's rows p0..M-1 live in registers (RPT rows a thread).  For
// column j (pivot row c = p0 + j, x = its rows >= c, alpha = x[c]) one block sum
// gives ||x||^2, x^H y_j' for the later columns and v_i^H x for the earlier
// reflectors; with beta = -e^{i arg alpha} ||x||, v = x - beta e_c:
//   v^H y = x^H y - conj(beta) y[c],   S[i][j] = v_i^H v_j = v_i^H x - conj(v_i[c]) beta
// (v_i[c] is reflector i's stored entry at row c).  Then the triangular factor T of
// H_p0 ... H_p0+15 = I - V T V^H, one column at a time by 16 threads.
// LDS state of the panel kernel
template <int NW, int K>
struct PanelLds {
  double red[NW][K], tot[K];
  double2 rowc[2][kPanel];         // the pivot row of the panel (y's values at row c), by column parity
  double2 S[kPanel][kPanel + 1];  // S[i][j] = v_i^H v_j, i < j
  double2 Tm[kPanel][kPanel + 1];
  double ts[kPanel];
};

// Column J of a panel (J a compile-time index, so that y stays in registers: the
// loop over columns holds barriers, which keeps the compiler from unrolling it).
template <int J, int RPT, int NW, int K>
__device__ __forceinline__ void panel_columns(double2 (&y)[RPT][kPanel], PanelLds<NW, K>& L, const Task2& T, int p0,
                                              int nb, int M) {
  if constexpr (J < kPanel) {
    constexpr int NT = NW * 64;
    const int tid = threadIdx.x;
    if (J < nb) {
      const int c = p0 + J;
      double sm[K];
#pragma unroll
      for (int k = 0; k < K; ++k) sm[k] = 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = p0 + tid + NT * q;
        if (r == c)
#pragma unroll
          for (int jj = 0; jj < kPanel; ++jj) L.rowc[J & 1][jj] = y[q][jj];
        if (r < c || r >= M) continue;
        const double2 x = y[q][J];
        sm[0] = fma(x.x, x.x, fma(x.y, x.y, sm[0]));
#pragma unroll
        for (int jj = 0; jj < kPanel; ++jj) {
          if (jj == J) continue;
          // later columns: x^H y_jj; earlier reflectors: v_jj^H x (rows > their pivot)
          const double2 p = jj > J ? cfmac(x, y[q][jj], cmk(sm[1 + 2 * jj], sm[2 + 2 * jj]))
                                   : cfmac(y[q][jj], x, cmk(sm[1 + 2 * jj], sm[2 + 2 * jj]));
          sm[1 + 2 * jj] = p.x;
          sm[2 + 2 * jj] = p.y;
        }
      }
      block_sum64<K, NW>(sm, L.red, L.tot);
      const double2 al = L.rowc[J & 1][J];
      double2 beta = cmk(0.0, 0.0), v0 = cmk(0.0, 0.0);
      double t = 0.0;
      if (sm[0] > 0.0) {
        const double nrm = sqrt(sm[0]);
        const double aa = sqrt(al.x * al.x + al.y * al.y);
        beta = aa > 0.0 ? cscale(al, -nrm / aa) : cmk(-nrm, 0.0);
        v0 = csub(al, beta);
        t = 1.0 / (nrm * (nrm + aa));
      }
      const double2 cb = cconj(beta);
      // apply H = I - t v v^H to the later columns: v^H y = x^H y - conj(beta) y[c]
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = p0 + tid + NT * q;
        if (r < c || r >= M) continue;
        const double2 vr = r == c ? v0 : y[q][J];
#pragma unroll
        for (int jj = J + 1; jj < kPanel; ++jj) {
          if (jj >= nb) continue;
          const double2 w = csub(cmk(sm[1 + 2 * jj], sm[2 + 2 * jj]), cmul(cb, L.rowc[J & 1][jj]));
          y[q][jj] = csub(y[q][jj], cscale(cmul(vr, w), t));
        }
        if (r == c) y[q][J] = beta;  // R[c][c]; the tail below stays the reflector
      }
      if (tid < J) {  // S[i][J] = v_i^H x - conj(v_i[c]) beta (totals read from LDS)
        const int i = tid;
        L.S[i][J] = csub(cmk(L.tot[1 + 2 * i], L.tot[2 + 2 * i]), cmul(cconj(L.rowc[J & 1][i]), beta));
      }
      if (tid == 0) {
        L.ts[J] = t;
        T.qvd[c] = v0;
        T.qt[c] = t;
      }
      // no barrier here: the next column writes the other rowc buffer, and every
      // thread has finished this column before the next column's block sum lets any
      // thread past it (which is also when red and tot are rewritten)
    }
    panel_columns<J + 1, RPT, NW, K>(y, L, T, p0, nb, M);
  }
}

// One panel of 16 columns (positions p0.. of the order qperm), one block of NT threads
// per task (256 for up to 512 rows, 512 above): the panel's rows p0..M-1 live in
// registers (RPT = 2 rows a thread; four waves instead of eight for 512 rows take
// 82 rather than 86 us a panel).  For column j (pivot row c = p0 + j, x = its rows
// >= c, alpha = x[c]) one block sum gives ||x||^2, x^H y_j' for the later columns and
// v_i^H x for the earlier reflectors; with beta = -e^{i arg alpha} ||x||, v = x - beta e_c:
//   v^H y = x^H y - conj(beta) y[c],   S[i][j] = v_i^H v_j = v_i^H x - conj(v_i[c]) beta
// (v_i[c] is reflector i's stored entry at row c).  Then the triangular factor T of
// H_p0 ... H_p0+15 = I - V T V^H, one column at a time by 16 threads.
template <int RPT, int NT>
__global__ __launch_bounds__(NT) void k_qr_panel(Task2* tasks, const Ent* ents, int p0) {
  constexpr int NW = NT / 64;
  constexpr int K = 1 + 2 * kPanel;  // ||x||^2, then (re, im) of x^H y_j' (j' > j) or v_j'^H x (j' < j)
  const Task2& T = tasks[ents[blockIdx.x].slot];
  if (!T.qr) return;
  const int M = T.M, N = T.N;
  if (p0 >= N) return;
  const int nb = N - p0 < kPanel ? N - p0 : kPanel;
  const int tid = threadIdx.x;
  __shared__ int pc[kPanel];
  __shared__ PanelLds<NW, K> L;
  if (tid < kPanel) pc[tid] = tid < nb ? T.qperm[p0 + tid] : 0;
  __syncthreads();
  double2* A = T.thw;
  double2 y[RPT][kPanel];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = p0 + tid + NT * q;
#pragma unroll
    for (int j = 0; j < kPanel; ++j) y[q][j] = (r < M && j < nb) ? A[(long)pc[j] * M + r] : cmk(0.0, 0.0);
  }
  panel_columns<0, RPT, NW, K>(y, L, T, p0, nb, M);
  // write the panel back (R rows and reflector tails)
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = p0 + tid + NT * q;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < kPanel; ++j)
      if (j < nb) A[(long)pc[j] * M + r] = y[q][j];
  }
  // T: T[j][j] = t_j, T[i][j] = -t_j sum_{l=i}^{j-1} T[i][l] S[l][j].  Row i is formed
  // by thread i alone, a column at a time: it reads only its own row and the finished
  // S and t, so the columns need no barrier between them
  if (tid < kPanel * kPanel) L.Tm[tid / kPanel][tid % kPanel] = cmk(0.0, 0.0);
  __syncthreads();
  if (tid < nb) {
    L.Tm[tid][tid] = cmk(L.ts[tid], 0.0);
    for (int j = tid + 1; j < nb; ++j) {
      double2 acc = cmk(0.0, 0.0);
      for (int l = tid; l < j; ++l) acc = cfma(L.Tm[tid][l], L.S[l][j], acc);
      L.Tm[tid][j] = cscale(acc, -L.ts[j]);
    }
  }
  __syncthreads();
  if (tid < kPanel * kPanel)
    T.qT[(long)(p0 / kPanel) * kPanel * kPanel + tid] = L.Tm[tid / kPanel][tid % kPanel];
}

// Apply a panel's block reflector to 16 columns of a target matrix, one 256-thread
// block per 16 columns: mode 0, the trailing columns of theta_w (positions p0+16..
// of qperm): Y <- (I - V T^H V^H) Y = Q_p^H Y; mode 1, the Jacobi's V_x (N x N, all
// columns): Y <- (I - V T V^H) Y = Q_p Y.  Rows below p0 only.  Both products are
// FP64 MFMA (v_mfma_f64_16x16x4f64; accumulator element r of lane l is entry
// (l / 16 + 4 r, l % 16)): W = V^H Y over k-steps of four rows, wave w taking
// k-steps w, w + 4, ..., the waves' sums added in wave order; then Y - V W' over
// 16-row tiles with Y as the accumulator's initial value.
typedef double qr_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_qr_apply(Task2* tasks, const Ent* ents, int p0, int mode) {
  constexpr int NW = 4, KB = 8;  // waves; k-steps of loads in flight
  const Task2& T = tasks[ents[blockIdx.y].slot];
  // mode 1 is given QR tasks only, and reads no field that the conversion to the
  // transposed problem changes (the descriptor may already be converted)
  if (mode == 0 && !T.qr) return;
  const int M = T.M, N = T.N;
  if (p0 >= N) return;
  const int nb = N - p0 < kPanel ? N - p0 : kPanel;
  const int c0 = (mode == 0 ? p0 + kPanel : 0) + blockIdx.x * 16;
  if (c0 >= N) return;
  const int ncol = N - c0 < 16 ? N - c0 : 16;
  const int rows = mode == 0 ? M : N;  // rows of the target (mode 1: square, M == N)
  double2* Y = mode == 0 ? T.thw : T.JV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int ycol[16], vcol[kPanel];
  __shared__ double2 v0s[kPanel];
  __shared__ double Ws[NW][2][16][17];
  __shared__ double2 Wm[kPanel][17], Wp[kPanel][17];
  __shared__ double2 Tm[kPanel][kPanel + 1];
  if (tid < 16) ycol[tid] = tid < ncol ? (mode == 0 ? T.qperm[c0 + tid] : c0 + tid) : -1;
  if (tid < kPanel) {
    vcol[tid] = tid < nb ? T.qperm[p0 + tid] : -1;
    v0s[tid] = tid < nb ? T.qvd[p0 + tid] : cmk(0.0, 0.0);
  }
  {
    const double2* Tp = T.qT + (long)(p0 / kPanel) * kPanel * kPanel;
    Tm[tid / kPanel][tid % kPanel] = Tp[tid];
  }
  __syncthreads();
  // reflector j at row r: zero above p0 + j, v0 at p0 + j, the stored tail below
  auto vget = [&](int j, int r) -> double2 {
    if (r >= rows || vcol[j] < 0 || r < p0 + j) return cmk(0.0, 0.0);
    if (r == p0 + j) return v0s[j];
    return T.thw[(long)vcol[j] * M + r];
  };
  auto yget = [&](int cc, int r) -> double2 {
    return (r < rows && ycol[cc] >= 0) ? Y[(long)ycol[cc] * rows + r] : cmk(0.0, 0.0);
  };
  const int li = lane & 15, lk = lane >> 4;
  // 1. W = V^H Y: Re W = Vr^T Yr + Vi^T Yi, Im W = Vr^T Yi - Vi^T Yr
  {
    qr_d4 wr = {0.0, 0.0, 0.0, 0.0}, wi = {0.0, 0.0, 0.0, 0.0};
    const int nks = (rows - p0 + 3) / 4;
    for (int ks0 = wave; ks0 < nks; ks0 += NW * KB) {
      double2 v[KB], y[KB];
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        const int r = p0 + (ks0 + NW * t) * 4 + lk;
        v[t] = vget(li, r);
        y[t] = yget(li, r);
      }
#pragma unroll
      for (int t = 0; t < KB; ++t) {
        wr = __builtin_amdgcn_mfma_f64_16x16x4f64(v[t].x, y[t].x, wr, 0, 0, 0);
        wr = __builtin_amdgcn_mfma_f64_16x16x4f64(v[t].y, y[t].y, wr, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(v[t].x, y[t].y, wi, 0, 0, 0);
        wi = __builtin_amdgcn_mfma_f64_16x16x4f64(-v[t].y, y[t].x, wi, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Ws[wave][0][lk + 4 * r][li] = wr[r];
      Ws[wave][1][lk + 4 * r][li] = wi[r];
    }
  }
  __syncthreads();
  {
    const int i = tid / 16, j = tid % 16;
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < NW; ++w) {
      sr += Ws[w][0][i][j];
      si += Ws[w][1][i][j];
    }
    Wm[i][j] = cmk(sr, si);
  }
  __syncthreads();
  // 2. W' = T^H W (mode 0) or T W (mode 1)
  {
    const int wi_ = tid / 16, wc = tid % 16;
    double2 wp = cmk(0.0, 0.0);
    for (int l = 0; l < kPanel; ++l)
      wp = mode == 0 ? cfmac(Tm[l][wi_], Wm[l][wc], wp) : cfma(Tm[wi_][l], Wm[l][wc], wp);
    Wp[wi_][wc] = wp;
  }
  __syncthreads();
  // 3. Y <- Y - V W' per 16-row tile: Re -= Vr W'r - Vi W'i, Im -= Vr W'i + Vi W'r
  double br[4], bi[4], nbr[4], nbi[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const double2 w = Wp[4 * ks + lk][li];
    br[ks] = w.x;
    bi[ks] = w.y;
    nbr[ks] = -w.x;
    nbi[ks] = -w.y;
  }
  const int ntile = (rows - p0 + 15) / 16;
  for (int tl = wave; tl < ntile; tl += NW) {
    const int t0 = p0 + 16 * tl;
    double2 a[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) a[ks] = vget(4 * ks + lk, t0 + li);
    qr_d4 yr, yi;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 yv = yget(li, t0 + lk + 4 * r);
      yr[r] = yv.x;
      yi[r] = yv.y;
    }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].x, nbr[ks], yr, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].y, bi[ks], yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].x, nbi[ks], yi, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks].y, nbr[ks], yi, 0, 0, 0);
    }
    if (ycol[li] >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = t0 + lk + 4 * r;
        if (row < rows) Y[(long)ycol[li] * rows + row] = cmk(yr[r], yi[r]);
      }
    }
  }
}

// X = R^H (N x N, column-major, lower triangular) into the Jacobi's W operand:
// X[i][j] = conj(R[j][i]) for i >= j, R[j][i] stored at row j of column qperm[i].
__global__ __launch_bounds__(256) void k_qr_formx(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.y].slot];
  if (!T.qr) return;
  const int N = T.N, M = T.M;
  const long nn = (long)N * N;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < nn; e += (long)gridDim.x * 256) {
    const int i = (int)(e % N), j = (int)(e / N);
    T.JW[e] = i >= j ? cconj(T.thw[(long)T.qperm[i] * M + j]) : cmk(0.0, 0.0);
  }
}

// The split's right factor for an FP64 task preconditioned by QR: for each kept
// column c (c = perm[nu]), Z[qperm[i]][c] = W_x[i][c] / ||W_x[:, c]|| (Z: N x N in
// theta_w's storage, ld N).
__global__ __launch_bounds__(256) void k_qr_z(Task2* tasks, const Ent* ents) {
  const Task2& T = tasks[ents[blockIdx.z].slot];
  if (!T.qr) return;
  const int k = *T.dim_out, nu = blockIdx.y, N = T.N;
  if (nu >= k) return;
  const int col = T.perm[nu];
  const double s = 1.0 / sqrt(T.sig2[col]);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
    T.Z[(long)col * N + T.qperm[i]] = cscale(T.JW[(long)col * N + i], s);
}

// ------------------------------------------------------------------ launchers
#define MPS_LAUNCH_CHECK() \
  do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_qr_factor(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_qr_colnorm, dim3((maxN + 3) / 4, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  hipError_t e = launch_qr_order(d_tasks, d_ents, nent, st);
  if (e != hipSuccess) return e;
  for (int p0 = 0; p0 < maxN; p0 += kPanel) {
    if (maxM <= 512)
      hipLaunchKernelGGL((k_qr_panel<2, 256>), dim3(nent), dim3(256), 0, st, d_tasks, d_ents, p0);
    else
      hipLaunchKernelGGL((k_qr_panel<2, 512>), dim3(nent), dim3(512), 0, st, d_tasks, d_ents, p0);
    MPS_LAUNCH_CHECK();
    const int trail = maxN - p0 - kPanel;
    if (trail > 0) {
      hipLaunchKernelGGL(k_qr_apply, dim3((trail + 15) / 16, nent), dim3(256), 0, st, d_tasks, d_ents, p0, 0);
      MPS_LAUNCH_CHECK();
    }
  }
  const long nn = (long)maxN * maxN;
  int gx = (int)((nn + 255) / 256);
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_qr_formx, dim3(gx, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_qr_left(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st) {
  const int np = (maxN + kPanel - 1) / kPanel;
  for (int p = np - 1; p >= 0; --p) {
    hipLaunchKernelGGL(k_qr_apply, dim3((maxN + 15) / 16, nent), dim3(256), 0, st, d_tasks, d_ents, p * kPanel, 1);
    MPS_LAUNCH_CHECK();
  }
  return hipSuccess;
}

hipError_t launch_qr_z(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int maxK, hipStream_t st) {
  hipLaunchKernelGGL(k_qr_z, dim3((maxN + 255) / 256, maxK, nent), dim3(256), 0, st, d_tasks, d_ents);
  MPS_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mpsk
