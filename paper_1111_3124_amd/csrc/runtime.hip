// Host runtime of the MPS gate-update library: handle lifetime, device memory,
// gate waves, the Jacobi sweep loop and the C ABI of include/mps.h.
//
// Bond dimensions live in a device table written by the truncation kernel; the
// host mirrors it after each wave (one small device-to-host copy), so that every
// launch is sized to the live shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mps.h"
#include "common.h"
#include "dd_kernels.h"
#include "launch.h"

using mpsk::Task1;
using mpsk::Task2;

namespace {

thread_local std::string g_create_error;

struct EvPair {
  hipEvent_t a, b;
  int cls;
  int n;
};

}  // namespace

struct mps_state {
  int n = 0, chi = 0, prec = MPS_PREC_FP64;
  double eps = 0.0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::vector<int> capx;  // capx[b+1] = capacity of bond b; capx[0] = capx[n] = 1
  std::vector<int> dimx;  // host mirror of the bond dims, same indexing
  int* d_dimx = nullptr;
  std::vector<double2*> B, Blo;  // per site, capx[s] * 2 * capx[s+1]
  double* d_lam = nullptr;       // (n+1) slots x chi; slot b+1 = bond b; slots 0, n = [1]
  double* d_lam_lo = nullptr;
  // options
  int max_sweeps = 40;
  int max_sweeps_dd = 16;
  int max_inner = 1;
  int block_width = 8;
  double tol_mult = 1.0;
  double rank_floor = 0x1p-44;
  double rank_floor_dd = 0x1p-96;
  bool timing = false;
  // workspace
  char* ws = nullptr;
  size_t ws_size = 0;
  char* h_stage = nullptr;  // pinned host staging (task arrays, readbacks)
  size_t h_stage_size = 0;
  char* d_small = nullptr;  // device task arrays + flags + stats
  size_t d_small_size = 0;
  // diagnostics
  mps_update_stats last{};
  std::string err;
  // timing
  std::vector<EvPair> pending;
  std::vector<hipEvent_t> evpool;
  double tms[8] = {0};
  long tcount[8] = {0};
};

namespace {

int fail(mps_state* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(h, call)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(h, e_ == hipErrorOutOfMemory ? MPS_ENOMEM : MPS_EDEVICE,                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                          \
  } while (0)

int bond_capacity(int n, int chi, int b) {
  // min(chi, 2^{b+1}, 2^{n-1-b})
  long c = chi;
  int l = b + 1, r = n - 1 - b;
  if (l < 31) c = std::min(c, 1L << l);
  if (r < 31) c = std::min(c, 1L << r);
  return (int)c;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

hipEvent_t ev_get(mps_state* h) {
  if (!h->evpool.empty()) {
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct Timed {
  mps_state* h;
  EvPair p{};
  bool on;
  // `launches` kernels are enqueued between the two events
  Timed(mps_state* hh, int cls, int launches = 1) : h(hh), on(hh->timing) {
    if (on) {
      p.a = ev_get(h);
      p.b = ev_get(h);
      p.cls = cls;
      p.n = launches;
      (void)hipEventRecord(p.a, h->stream);
    }
  }
  ~Timed() {
    if (on) {
      (void)hipEventRecord(p.b, h->stream);
      h->pending.push_back(p);
    }
  }
};

// after a synchronisation: fold finished event pairs into the per-class totals
void harvest_timing(mps_state* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->tms[p.cls] += ms;
      h->tcount[p.cls] += p.n;
    }
    h->evpool.push_back(p.a);
    h->evpool.push_back(p.b);
  }
  h->pending.clear();
}

int ensure_ws(mps_state* h, size_t bytes) {
  if (bytes <= h->ws_size) return MPS_OK;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->ws) HIPCHK(h, hipFree(h->ws));
  h->ws = nullptr;
  h->ws_size = 0;
  size_t want = std::max(bytes, h->ws_size * 3 / 2);
  HIPCHK(h, hipMalloc((void**)&h->ws, want));
  h->ws_size = want;
  return MPS_OK;
}

int ensure_small(mps_state* h, size_t bytes) {
  if (bytes <= h->d_small_size && bytes <= h->h_stage_size) return MPS_OK;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  size_t want = std::max<size_t>(bytes, 1 << 16);
  if (bytes > h->d_small_size) {
    if (h->d_small) HIPCHK(h, hipFree(h->d_small));
    h->d_small = nullptr;
    HIPCHK(h, hipMalloc((void**)&h->d_small, want));
    h->d_small_size = want;
  }
  if (bytes > h->h_stage_size) {
    if (h->h_stage) HIPCHK(h, hipHostFree(h->h_stage));
    h->h_stage = nullptr;
    HIPCHK(h, hipHostMalloc((void**)&h->h_stage, want, hipHostMallocDefault));
    h->h_stage_size = want;
  }
  return MPS_OK;
}

bool finite_gate(int k, const double* U) {
  const int nd = 2 << (2 * k);
  for (int i = 0; i < nd; ++i)
    if (!std::isfinite(U[i])) return false;
  return true;
}

int validate_gate(mps_state* h, int first, int k, const double* U, const double* Ulo) {
  if (k < 1 || k > 3) return fail(h, MPS_EINVAL, "k must be 1, 2 or 3");
  if (first < 0 || first + k > h->n) return fail(h, MPS_EINVAL, "gate sites out of range");
  if (!U) return fail(h, MPS_EINVAL, "null gate matrix");
  if (!finite_gate(k, U) || (Ulo && !finite_gate(k, Ulo)))
    return fail(h, MPS_ENONFINITE, "gate matrix has a NaN or infinite entry");
  return MPS_OK;
}

struct GateRef {
  int first, k;
  const double* U;
  const double* Ulo;
};

// ------------------------------------------------------------------ single-site wave
int run_wave1(mps_state* h, const std::vector<GateRef>& g1) {
  if (g1.empty()) return MPS_OK;
  const int nt = (int)g1.size();
  int rc = ensure_small(h, align_up(sizeof(Task1) * nt));
  if (rc) return rc;
  Task1* ht = (Task1*)h->h_stage;
  long maxel = 0;
  for (int i = 0; i < nt; ++i) {
    const int s = g1[i].first;
    Task1 t{};
    t.B = h->B[s];
    t.B_lo = h->Blo.empty() ? nullptr : h->Blo[s];
    t.ld = h->capx[s + 1];
    t.a = h->dimx[s];
    t.b = h->dimx[s + 1];
    for (int e = 0; e < 4; ++e) {
      t.U[e] = make_double2(g1[i].U[2 * e], g1[i].U[2 * e + 1]);
      t.U_lo[e] = g1[i].Ulo ? make_double2(g1[i].Ulo[2 * e], g1[i].Ulo[2 * e + 1]) : make_double2(0, 0);
    }
    ht[i] = t;
    maxel = std::max(maxel, (long)t.a * t.b);
  }
  Task1* dt = (Task1*)h->d_small;
  HIPCHK(h, hipMemcpyAsync(dt, ht, sizeof(Task1) * nt, hipMemcpyHostToDevice, h->stream));
  {
    Timed tm(h, 4);
    hipError_t e = (h->prec == MPS_PREC_DD) ? mpsk::launch_gate1_dd(dt, nt, maxel, h->stream)
                                            : mpsk::launch_gate1(dt, nt, maxel, h->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("gate1: ") + hipGetErrorString(e));
  }
  // the staging buffer is reused by the next wave: wait for the copy
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  h->last.splits = 0;
  return MPS_OK;
}

// ------------------------------------------------------------------ two-site wave
int run_wave2(mps_state* h, const std::vector<GateRef>& g2) {
  if (g2.empty()) return MPS_OK;
  const int nt = (int)g2.size();
  const bool dd = h->prec == MPS_PREC_DD;
  // workspace layout per task
  std::vector<size_t> off(nt + 1, 0);
  int maxM = 0, maxN = 0;
  for (int i = 0; i < nt; ++i) {
    const int s = g2[i].first;
    const int M = 2 * h->dimx[s], N = 2 * h->dimx[s + 2];
    maxM = std::max(maxM, M);
    maxN = std::max(maxN, N);
    size_t cplx = (size_t)2 * M * N + (size_t)N * N;
    size_t bytes = align_up(cplx * sizeof(double2)) * (dd ? 2 : 1) + align_up(N * sizeof(double)) * (dd ? 2 : 1) +
                   align_up(N * sizeof(int)) + (dd ? 2 * align_up((size_t)N * N * sizeof(double2)) : 0);
    off[i + 1] = off[i] + bytes;
  }
  int rc = ensure_ws(h, off[nt]);
  if (rc) return rc;
  // small device area: tasks | flags (3/task) | stats (8/task) | fro2 (1/task) | dimx copy
  const size_t o_tasks = 0;
  const size_t o_flags = align_up(sizeof(Task2) * nt);
  const size_t o_stats = o_flags + align_up(sizeof(int) * 3 * nt);
  const size_t o_fro = o_stats + align_up(sizeof(double) * 8 * nt);
  const size_t o_dims = o_fro + align_up(sizeof(double) * nt);
  const size_t o_end = o_dims + align_up(sizeof(int) * (h->n + 1));
  rc = ensure_small(h, o_end);
  if (rc) return rc;
  Task2* ht = (Task2*)(h->h_stage + o_tasks);
  Task2* dt = (Task2*)(h->d_small + o_tasks);
  int* d_flags = (int*)(h->d_small + o_flags);
  double* d_stats = (double*)(h->d_small + o_stats);
  double* d_fro = (double*)(h->d_small + o_fro);
  for (int i = 0; i < nt; ++i) {
    const int s = g2[i].first;
    Task2 t{};
    t.Bl = h->B[s];
    t.Br = h->B[s + 1];
    t.Bl_lo = dd ? h->Blo[s] : nullptr;
    t.Br_lo = dd ? h->Blo[s + 1] : nullptr;
    t.ldl = h->capx[s + 1];
    t.ldr = h->capx[s + 2];
    t.a = h->dimx[s];
    t.b = h->dimx[s + 1];
    t.c = h->dimx[s + 2];
    t.M = 2 * t.a;
    t.N = 2 * t.c;
    t.lamL = h->d_lam + (size_t)s * h->chi;
    t.lamL_lo = dd ? h->d_lam_lo + (size_t)s * h->chi : nullptr;
    t.lamS = h->d_lam + (size_t)(s + 1) * h->chi;
    t.lamS_lo = dd ? h->d_lam_lo + (size_t)(s + 1) * h->chi : nullptr;
    t.dim_out = h->d_dimx + s + 1;
    for (int e = 0; e < 16; ++e) {
      t.U[e] = make_double2(g2[i].U[2 * e], g2[i].U[2 * e + 1]);
      t.U_lo[e] = (dd && g2[i].Ulo) ? make_double2(g2[i].Ulo[2 * e], g2[i].Ulo[2 * e + 1]) : make_double2(0, 0);
    }
    char* w = h->ws + off[i];
    const size_t MN = (size_t)t.M * t.N, NN = (size_t)t.N * t.N;
    t.thu = (double2*)w;
    t.thw = t.thu + MN;
    t.V = t.thw + MN;
    w += align_up((2 * MN + NN) * sizeof(double2));
    if (dd) {
      t.thu_lo = (double2*)w;
      t.thw_lo = t.thu_lo + MN;
      t.V_lo = t.thw_lo + MN;
      w += align_up((2 * MN + NN) * sizeof(double2));
      t.aux1 = (double2*)w;
      w += align_up(NN * sizeof(double2));
      t.aux2 = (double2*)w;
      w += align_up(NN * sizeof(double2));
    }
    t.sig2 = (double*)w;
    w += align_up(t.N * sizeof(double));
    if (dd) {
      t.sig2_lo = (double*)w;
      w += align_up(t.N * sizeof(double));
    }
    t.perm = (int*)w;
    t.flags = d_flags + 3 * i;
    t.stats = d_stats + 8 * i;
    t.fro2 = d_fro + i;
    ht[i] = t;
  }
  HIPCHK(h, hipMemcpyAsync(dt, ht, sizeof(Task2) * nt, hipMemcpyHostToDevice, h->stream));
  hipError_t e;
  {
    Timed tm(h, 0);
    e = mpsk::launch_prep2(dt, nt, maxN, h->stream);
    if (e == hipSuccess)
      e = dd ? mpsk::launch_theta2_dd(dt, nt, maxM, maxN, h->stream)
             : mpsk::launch_theta2(dt, nt, maxM, maxN, h->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("theta: ") + hipGetErrorString(e));
  }
  // Jacobi sweeps on the FP64 (hi) part of theta_w
  const int bw = h->block_width;
  const int nb = (maxN + bw - 1) / bw;
  const int nsteps = nb + (nb & 1) - 1;
  int* hflags = (int*)(h->h_stage + o_flags);
  int sweeps = 0;
  bool converged = false;
  for (int sw = 0; sw < h->max_sweeps; ++sw) {
    {
      Timed tm(h, 1, nsteps);
      for (int st = 0; st < nsteps; ++st) {
        e = mpsk::launch_jacobi_step(dt, nt, maxN, bw, st, sw, h->tol_mult, h->max_inner, h->stream);
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("jacobi: ") + hipGetErrorString(e));
      }
    }
    HIPCHK(h, hipMemcpyAsync(hflags, d_flags, sizeof(int) * 3 * nt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    sweeps = sw + 1;
    bool any = false;
    for (int i = 0; i < nt; ++i) any |= hflags[3 * i + sw % 3] != 0;
    if (!any) {
      converged = true;
      break;
    }
  }
  int dd_sweeps = 0;
  bool dd_conv = true;
  if (dd) {
    Timed tm(h, 6);
    int r2 = mpsk::run_dd_refine(dt, nt, maxM, maxN, h->max_sweeps_dd, h->max_inner, h->tol_mult, hflags, d_flags,
                                 h->stream, &dd_sweeps, &dd_conv);
    if (r2 != 0) return fail(h, MPS_EDEVICE, "dd refinement failed");
  }
  {
    Timed tm(h, 2);
    e = dd ? mpsk::launch_truncate_dd(dt, nt, h->chi, h->eps, h->rank_floor_dd, h->stream)
           : mpsk::launch_truncate(dt, nt, h->chi, h->eps, h->rank_floor, h->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("truncate: ") + hipGetErrorString(e));
  }
  {
    Timed tm(h, 3);
    const int maxK = std::min(h->chi, std::min(maxM, maxN));
    e = dd ? mpsk::launch_split_dd(dt, nt, maxM, maxN, maxK, h->stream)
           : mpsk::launch_split(dt, nt, maxM, maxN, maxK, h->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("split: ") + hipGetErrorString(e));
  }
  double* hstats = (double*)(h->h_stage + o_stats);
  HIPCHK(h, hipMemcpyAsync(hstats, d_stats, sizeof(double) * 8 * nt, hipMemcpyDeviceToHost, h->stream));
  std::vector<int> nd(h->n + 1);
  HIPCHK(h, hipMemcpyAsync(h->h_stage + o_dims, h->d_dimx, sizeof(int) * (h->n + 1), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::memcpy(nd.data(), h->h_stage + o_dims, sizeof(int) * (h->n + 1));
  h->dimx = nd;
  harvest_timing(h);
  const double* st = hstats + 8 * (nt - 1);
  h->last.W = st[0];
  h->last.w = st[1];
  h->last.gap = st[2];
  h->last.epsdist = st[3];
  h->last.k = (int)st[4];
  h->last.rank = (int)st[5];
  h->last.sweeps = sweeps;
  h->last.dd_sweeps = dd_sweeps;
  h->last.splits = 1;
  // a dd handle's result is the dd polish: its convergence is what counts
  if (dd ? !dd_conv : !converged) return fail(h, MPS_ENOCONV, "Jacobi sweep limit reached");
  return MPS_OK;
}

// Split a gate list into waves of gates on disjoint sites and run them.
int run_gates(mps_state* h, const std::vector<GateRef>& gates) {
  size_t i = 0;
  int status = MPS_OK;
  while (i < gates.size()) {
    std::vector<char> busy(h->n, 0);
    std::vector<GateRef> w1, w2, w3;
    size_t j = i;
    for (; j < gates.size(); ++j) {
      const GateRef& g = gates[j];
      bool clash = false;
      for (int q = g.first; q < g.first + g.k; ++q) clash |= busy[q] != 0;
      if (clash) break;
      for (int q = g.first; q < g.first + g.k; ++q) busy[q] = 1;
      (g.k == 1 ? w1 : g.k == 2 ? w2 : w3).push_back(g);
    }
    int rc = run_wave1(h, w1);
    if (rc) return rc;
    rc = run_wave2(h, w2);
    if (rc == MPS_ENOCONV) status = rc;
    else if (rc) return rc;
    if (!w3.empty()) return fail(h, MPS_ESTATE, "three-site gates are not available in this build");
    i = j;
  }
  return status;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* mps_version(void) { return "mps-mi355x 0.1 (gfx950)"; }

const char* mps_last_error(mps_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

mps_handle mps_create_ex(int n, int chi_max, double eps, int prec, void* hip_stream) {
  g_create_error.clear();
  if (n < 1 || chi_max < 1 || !(eps >= 0) || !std::isfinite(eps) || (prec != MPS_PREC_FP64 && prec != MPS_PREC_DD)) {
    g_create_error = "mps_create: need n >= 1, chi_max >= 1, finite eps >= 0, prec FP64 or DD";
    return nullptr;
  }
  if (prec == MPS_PREC_DD && !mpsk::dd_available()) {
    g_create_error = "mps_create: double-double precision is not available in this build";
    return nullptr;
  }
  if (chi_max > 2048) {
    g_create_error = "mps_create: chi_max above 2048 is not supported";
    return nullptr;
  }
  mps_state* h = new mps_state();
  h->n = n;
  h->chi = chi_max;
  h->eps = eps;
  h->prec = prec;
  auto bail = [&](const char* what, hipError_t e) {
    g_create_error = std::string(what) + ": " + hipGetErrorString(e);
    mps_destroy(h);
    return (mps_handle) nullptr;
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return bail("hipGetDevice", e);
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail("hipStreamCreate", e);
    h->own_stream = true;
  }
  h->capx.assign(n + 1, 1);
  for (int b = 0; b + 1 < n; ++b) h->capx[b + 1] = bond_capacity(n, chi_max, b);
  h->dimx.assign(n + 1, 1);
  e = hipMalloc((void**)&h->d_dimx, sizeof(int) * (n + 1));
  if (e != hipSuccess) return bail("hipMalloc", e);
  const bool dd = prec == MPS_PREC_DD;
  h->B.assign(n, nullptr);
  if (dd) h->Blo.assign(n, nullptr);
  for (int s = 0; s < n; ++s) {
    size_t el = (size_t)h->capx[s] * 2 * h->capx[s + 1];
    e = hipMalloc((void**)&h->B[s], el * sizeof(double2));
    if (e != hipSuccess) return bail("hipMalloc", e);
    if (dd) {
      e = hipMalloc((void**)&h->Blo[s], el * sizeof(double2));
      if (e != hipSuccess) return bail("hipMalloc", e);
    }
  }
  size_t lam_el = (size_t)(n + 1) * chi_max;
  e = hipMalloc((void**)&h->d_lam, lam_el * sizeof(double));
  if (e != hipSuccess) return bail("hipMalloc", e);
  if (dd) {
    e = hipMalloc((void**)&h->d_lam_lo, lam_el * sizeof(double));
    if (e != hipSuccess) return bail("hipMalloc", e);
  }
  // |0...0>: B_s[0][0][0] = 1, B_s[0][1][0] = 0, all V_s = [1]
  std::vector<double> lam(lam_el, 0.0);
  for (int sl = 0; sl <= n; ++sl) lam[(size_t)sl * chi_max] = 1.0;
  e = hipMemcpy(h->d_lam, lam.data(), lam_el * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail("hipMemcpy", e);
  if (dd) {
    e = hipMemset(h->d_lam_lo, 0, lam_el * sizeof(double));
    if (e != hipSuccess) return bail("hipMemset", e);
  }
  for (int s = 0; s < n; ++s) {
    size_t el = (size_t)h->capx[s] * 2 * h->capx[s + 1];
    std::vector<double2> z(el, make_double2(0, 0));
    z[0] = make_double2(1.0, 0.0);
    e = hipMemcpy(h->B[s], z.data(), el * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail("hipMemcpy", e);
    if (dd) {
      e = hipMemset(h->Blo[s], 0, el * sizeof(double2));
      if (e != hipSuccess) return bail("hipMemset", e);
    }
  }
  e = hipMemcpy(h->d_dimx, h->dimx.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail("hipMemcpy", e);
  return h;
}

mps_handle mps_create(int n, int chi_max, double eps) {
  return mps_create_ex(n, chi_max, eps, MPS_PREC_FP64, nullptr);
}

int mps_destroy(mps_handle h) {
  if (!h) return MPS_EINVAL;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (auto p : h->B) if (p) (void)hipFree(p);
  for (auto p : h->Blo) if (p) (void)hipFree(p);
  if (h->d_lam) (void)hipFree(h->d_lam);
  if (h->d_lam_lo) (void)hipFree(h->d_lam_lo);
  if (h->d_dimx) (void)hipFree(h->d_dimx);
  if (h->ws) (void)hipFree(h->ws);
  if (h->d_small) (void)hipFree(h->d_small);
  if (h->h_stage) (void)hipHostFree(h->h_stage);
  for (auto& p : h->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : h->evpool) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return MPS_OK;
}

int mps_apply_gates(mps_handle h, int count, const int* first, const int* k, const double* U, const double* U_lo) {
  if (!h) return MPS_EINVAL;
  if (count < 0 || (count > 0 && (!first || !k || !U))) return fail(h, MPS_EINVAL, "bad gate list");
  std::vector<GateRef> gates;
  gates.reserve(count);
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const double* lo = U_lo ? U_lo + off : nullptr;
    int rc = validate_gate(h, first[i], k[i], U + off, h->prec == MPS_PREC_DD ? lo : nullptr);
    if (rc) return rc;
    gates.push_back(GateRef{first[i], k[i], U + off, h->prec == MPS_PREC_DD ? lo : nullptr});
    off += (size_t)2 << (2 * k[i]);
  }
  return run_gates(h, gates);
}

int mps_apply_gate(mps_handle h, int first, int k, const double* U) {
  return mps_apply_gates(h, 1, &first, &k, U, nullptr);
}

int mps_apply_gate_dd(mps_handle h, int first, int k, const double* U_hi, const double* U_lo) {
  return mps_apply_gates(h, 1, &first, &k, U_hi, U_lo);
}

int mps_bond_dim(mps_handle h, int bond, int* m) {
  if (!h || !m) return MPS_EINVAL;
  if (bond < 0 || bond > h->n - 2) return fail(h, MPS_EINVAL, "bond out of range");
  *m = h->dimx[bond + 1];
  return MPS_OK;
}

int mps_schmidt_dd(mps_handle h, int bond, double* lam_hi, double* lam_lo, int cap, int* m) {
  if (!h || !lam_hi || !m) return MPS_EINVAL;
  if (bond < 0 || bond > h->n - 2) return fail(h, MPS_EINVAL, "bond out of range");
  const int mm = h->dimx[bond + 1];
  *m = mm;
  if (cap < mm) return fail(h, MPS_ERANGE, "Schmidt buffer too small");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(lam_hi, h->d_lam + (size_t)(bond + 1) * h->chi, sizeof(double) * mm, hipMemcpyDeviceToHost));
  if (lam_lo) {
    if (h->d_lam_lo)
      HIPCHK(h, hipMemcpy(lam_lo, h->d_lam_lo + (size_t)(bond + 1) * h->chi, sizeof(double) * mm,
                          hipMemcpyDeviceToHost));
    else
      std::memset(lam_lo, 0, sizeof(double) * mm);
  }
  return MPS_OK;
}

int mps_schmidt(mps_handle h, int bond, double* lam, int cap, int* m) {
  return mps_schmidt_dd(h, bond, lam, nullptr, cap, m);
}

int mps_amplitudes(mps_handle h, int count, const unsigned char* bits, double* out) {
  if (!h || count < 0 || (count > 0 && (!bits || !out))) return MPS_EINVAL;
  if (count == 0) return MPS_OK;
  for (long i = 0; i < (long)count * h->n; ++i)
    if (bits[i] > 1) return fail(h, MPS_EINVAL, "bits must be 0 or 1");
  for (int s = 0; s <= h->n; ++s)
    if (h->dimx[s] > 1024) return fail(h, MPS_ERANGE, "amplitude kernel supports bond dims up to 1024");
  const bool dd = h->prec == MPS_PREC_DD;
  const size_t nbits = align_up((size_t)count * h->n);
  const size_t o_ptr = nbits, o_ld = o_ptr + align_up(sizeof(void*) * 2 * h->n), o_out = o_ld + align_up(sizeof(int) * h->n);
  const size_t outb = (size_t)count * sizeof(double2) * (dd ? 2 : 1);
  int rc = ensure_small(h, o_out + align_up(outb));
  if (rc) return rc;
  char* hs = h->h_stage;
  std::memcpy(hs, bits, (size_t)count * h->n);
  const double2** hp = (const double2**)(hs + o_ptr);
  for (int s = 0; s < h->n; ++s) {
    hp[s] = h->B[s];
    hp[h->n + s] = dd ? h->Blo[s] : nullptr;
  }
  int* hld = (int*)(hs + o_ld);
  for (int s = 0; s < h->n; ++s) hld[s] = h->capx[s + 1];
  HIPCHK(h, hipMemcpyAsync(h->d_small, hs, o_out, hipMemcpyHostToDevice, h->stream));
  mpsk::AmpArgs a{};
  a.B = (const double2* const*)(h->d_small + o_ptr);
  a.ld = (const int*)(h->d_small + o_ld);
  a.dimx = h->d_dimx;
  a.n = h->n;
  a.bits = (const unsigned char*)h->d_small;
  a.out = (double2*)(h->d_small + o_out);
  {
    Timed tm(h, 5);
    hipError_t e = dd ? mpsk::launch_amplitude_dd(a, (const double2* const*)(h->d_small + o_ptr) + h->n, count, h->stream)
                      : mpsk::launch_amplitude(a, count, h->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("amplitude: ") + hipGetErrorString(e));
  }
  HIPCHK(h, hipMemcpyAsync(hs + o_out, h->d_small + o_out, outb, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  std::memcpy(out, hs + o_out, outb);
  return MPS_OK;
}

int mps_amplitude(mps_handle h, const unsigned char* bits, double out[2]) {
  if (!h) return MPS_EINVAL;
  if (h->prec == MPS_PREC_DD) {
    double o4[4];
    int rc = mps_amplitudes(h, 1, bits, o4);
    if (rc) return rc;
    out[0] = o4[0] + o4[1];
    out[1] = o4[2] + o4[3];
    return MPS_OK;
  }
  return mps_amplitudes(h, 1, bits, out);
}

int mps_amplitude_dd(mps_handle h, const unsigned char* bits, double out[4]) {
  if (!h) return MPS_EINVAL;
  if (h->prec != MPS_PREC_DD) {
    double o2[2];
    int rc = mps_amplitudes(h, 1, bits, o2);
    if (rc) return rc;
    out[0] = o2[0]; out[1] = 0.0; out[2] = o2[1]; out[3] = 0.0;
    return MPS_OK;
  }
  return mps_amplitudes(h, 1, bits, out);
}

int mps_stats(mps_handle h, mps_update_stats* s) {
  if (!h || !s) return MPS_EINVAL;
  *s = h->last;
  return MPS_OK;
}

int mps_load(mps_handle h, const int* dims, const double* const* B, const double* const* B_lo,
             const double* const* lam, const double* const* lam_lo) {
  if (!h || !B || (h->n > 1 && (!dims || !lam))) return MPS_EINVAL;
  const bool dd = h->prec == MPS_PREC_DD;
  std::vector<int> nd(h->n + 1, 1);
  for (int b = 0; b + 1 < h->n; ++b) {
    if (dims[b] < 1 || dims[b] > h->capx[b + 1]) return fail(h, MPS_ERANGE, "bond dim above the bond's capacity");
    nd[b + 1] = dims[b];
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int s = 0; s < h->n; ++s) {
    const int a = nd[s], b = nd[s + 1], ld = h->capx[s + 1];
    for (int plane = 0; plane < (dd ? 2 : 1); ++plane) {
      const double* src = plane ? (B_lo ? B_lo[s] : nullptr) : B[s];
      double2* dst = plane ? h->Blo[s] : h->B[s];
      if (!src) {
        HIPCHK(h, hipMemset(dst, 0, sizeof(double2) * (size_t)h->capx[s] * 2 * ld));
        continue;
      }
      HIPCHK(h, hipMemcpy2D(dst, sizeof(double2) * ld, src, sizeof(double2) * b, sizeof(double2) * b, (size_t)2 * a,
                            hipMemcpyHostToDevice));
    }
  }
  for (int b = 0; b + 1 < h->n; ++b) {
    HIPCHK(h, hipMemcpy(h->d_lam + (size_t)(b + 1) * h->chi, lam[b], sizeof(double) * nd[b + 1], hipMemcpyHostToDevice));
    if (dd) {
      if (lam_lo)
        HIPCHK(h, hipMemcpy(h->d_lam_lo + (size_t)(b + 1) * h->chi, lam_lo[b], sizeof(double) * nd[b + 1],
                            hipMemcpyHostToDevice));
      else
        HIPCHK(h, hipMemset(h->d_lam_lo + (size_t)(b + 1) * h->chi, 0, sizeof(double) * nd[b + 1]));
    }
  }
  HIPCHK(h, hipMemcpy(h->d_dimx, nd.data(), sizeof(int) * (h->n + 1), hipMemcpyHostToDevice));
  h->dimx = nd;
  return MPS_OK;
}

int mps_get_site(mps_handle h, int s, double* hi, double* lo, long cap_doubles) {
  if (!h || !hi) return MPS_EINVAL;
  if (s < 0 || s >= h->n) return fail(h, MPS_EINVAL, "site out of range");
  const int a = h->dimx[s], b = h->dimx[s + 1], ld = h->capx[s + 1];
  if (cap_doubles < (long)a * 2 * b * 2) return fail(h, MPS_ERANGE, "site buffer too small");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy2D(hi, sizeof(double2) * b, h->B[s], sizeof(double2) * ld, sizeof(double2) * b, (size_t)2 * a,
                        hipMemcpyDeviceToHost));
  if (lo) {
    if (h->prec == MPS_PREC_DD)
      HIPCHK(h, hipMemcpy2D(lo, sizeof(double2) * b, h->Blo[s], sizeof(double2) * ld, sizeof(double2) * b,
                            (size_t)2 * a, hipMemcpyDeviceToHost));
    else
      std::memset(lo, 0, sizeof(double) * (size_t)a * 2 * b * 2);
  }
  return MPS_OK;
}

int mps_set_option(mps_handle h, int key, double value) {
  if (!h) return MPS_EINVAL;
  switch (key) {
    case MPS_OPT_MAX_SWEEPS:
      if (!(value >= 1 && value <= 1000)) return fail(h, MPS_EINVAL, "max_sweeps out of range");
      h->max_sweeps = (int)value;
      h->max_sweeps_dd = (int)value;
      return MPS_OK;
    case MPS_OPT_JACOBI_TOL:
      if (!(value > 0 && value <= 1e6)) return fail(h, MPS_EINVAL, "jacobi tol out of range");
      h->tol_mult = value;
      return MPS_OK;
    case MPS_OPT_KERNEL_TIMING:
      h->timing = value != 0;
      return MPS_OK;
    case MPS_OPT_BLOCK_WIDTH:
      if (!(value == 4 || value == 8 || value == 16)) return fail(h, MPS_EINVAL, "block width must be 4, 8 or 16");
      h->block_width = (int)value;
      return MPS_OK;
    case MPS_OPT_MAX_INNER:
      if (!(value >= 1 && value <= 64)) return fail(h, MPS_EINVAL, "inner sweep limit out of range");
      h->max_inner = (int)value;
      return MPS_OK;
    case MPS_OPT_RANK_FLOOR:
      if (!(value >= 0 && value < 1)) return fail(h, MPS_EINVAL, "rank floor out of range");
      if (h->prec == MPS_PREC_DD) h->rank_floor_dd = value; else h->rank_floor = value;
      return MPS_OK;
    default:
      return fail(h, MPS_EINVAL, "unknown option");
  }
}

int mps_sync(mps_handle h) {
  if (!h) return MPS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  return MPS_OK;
}

int mps_kernel_time(mps_handle h, int cls, double* ms, long* launches, int reset) {
  if (!h || cls < 0 || cls >= 8) return MPS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  if (ms) *ms = h->tms[cls];
  if (launches) *launches = h->tcount[cls];
  if (reset) { h->tms[cls] = 0; h->tcount[cls] = 0; }
  return MPS_OK;
}

}  // extern "C"
