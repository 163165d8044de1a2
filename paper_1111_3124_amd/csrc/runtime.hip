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
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mps.h"
#include "common.h"
#include "dd_kernels.h"
#include "kernels3.h"
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
  int max_slots = 32;
  double tol_mult = 1.0;
  double rank_floor = 0x1p-44;
  double rank_floor_dd = 0x1p-96;
  bool timing = false;
  bool debug_sweeps = false;  // MPS_DEBUG_SWEEPS=1: print per-update sweep counts
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
  long slot_sweeps = 0, slot_sweeps_dd = 0;  // update-sweeps executed (FP64, dd polish)
  long long* d_phase = nullptr;               // MPS_DEBUG_PHASES=1: step phase stamps
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

// ------------------------------------------------------------------ update scheduler
// Continuous batching of gate updates.  Each two-site split occupies a slot (task
// descriptor + workspace).  One scheduler tick:
//   1. admit queued gates whose sites are free and not claimed by an earlier queued
//      gate (gates on disjoint sites commute, so queue order is kept where it
//      matters): a single-site gate runs at once; a two-site gate takes a slot and
//      gets its prep + theta launch; a three-site gate takes a slot for its first
//      split (s | s+1 s+2) and reserves a second one for its second split;
//   2. one Jacobi sweep for every slot still iterating (FP64 sweeps, or dd polish
//      sweeps after the FP64 iteration of a dd handle has converged);
//   3. read the rotation flags; converged slots are truncated and split at once and
//      their new bond dimensions read back.  A finished first split of a three-site
//      gate hands Z1_k^H, weighted by its new Schmidt values, to the reserved slot as
//      the theta of the second split; any other finished slot frees its sites.
// A slow update never holds back updates that do not depend on it.
struct Slot {
  int state = 0;  // 0 free, 1 FP64 Jacobi, 2 dd polish, 3 ready to finalise, 5 reserved
  int kind = 0;   // 0 two-site, 1 three-site first split, 2 three-site second split
  int gate = -1;
  int partner = -1;  // kind 1: the reserved slot of the second split
  int sweep = 0;
  int fp64_sweeps = 0, dd_sweeps = 0;
  bool fp64_conv = false, conv = false;
  int M = 0, N = 0;
};

struct SchedBufs {
  int S = 0;
  size_t slot_bytes = 0;
  // offsets in the small device / pinned areas
  size_t o_tasks = 0, o_flags = 0, o_stats = 0, o_fro = 0, o_dims = 0, o_u8 = 0, o_ents = 0, o_end = 0;
  static constexpr int kLists = 9;  // new2, new3, jacobi, dd, dd-enter, final, final3, mid, gate1
};

size_t slot_workspace_bytes(const mps_state* h, int Mcap, int Ncap, int t1cap) {
  const bool dd = h->prec == MPS_PREC_DD;
  const size_t MN = (size_t)Mcap * Ncap, NN = (size_t)Ncap * Ncap;
  size_t b = align_up((2 * MN + NN) * sizeof(double2)) * (dd ? 2 : 1);
  if (dd) b += 2 * align_up(NN * sizeof(double2));
  b += align_up(Ncap * sizeof(double)) * (dd ? 2 : 1) + align_up(Ncap * sizeof(int));
  b += align_up((size_t)t1cap * sizeof(double2)) * (dd ? 2 : 1);
  return b;
}

// workspace pointers of a task whose theta is M x N, carved from the slot region w
void carve(mps_state* h, Task2& t, char* w, int* d_flags, double* d_stats, double* d_fro, int slot) {
  const bool dd = h->prec == MPS_PREC_DD;
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
  w += align_up(t.N * sizeof(int));
  if (t.B3) {
    const size_t t1 = (size_t)4 * t.a * t.c;
    t.T1 = (double2*)w;
    w += align_up(t1 * sizeof(double2));
    if (dd) t.T1_lo = (double2*)w;
  }
  t.flags = d_flags + 3 * slot;
  t.stats = d_stats + 8 * slot;
  t.fro2 = d_fro + slot;
}

// the two-site split between sites s and s+1 with bond dims a | (b) | c
void setup_split(mps_state* h, Task2& t, int s, int a, int b, int c) {
  const bool dd = h->prec == MPS_PREC_DD;
  t = Task2{};
  t.Bl = h->B[s];
  t.Br = h->B[s + 1];
  t.Bl_lo = dd ? h->Blo[s] : nullptr;
  t.Br_lo = dd ? h->Blo[s + 1] : nullptr;
  t.ldl = h->capx[s + 1];
  t.ldr = h->capx[s + 2];
  t.a = a;
  t.b = b;
  t.c = c;
  t.M = 2 * a;
  t.N = 2 * c;
  t.lamL = h->d_lam + (size_t)s * h->chi;
  t.lamL_lo = dd ? h->d_lam_lo + (size_t)s * h->chi : nullptr;
  t.lamS = h->d_lam + (size_t)(s + 1) * h->chi;
  t.lamS_lo = dd ? h->d_lam_lo + (size_t)(s + 1) * h->chi : nullptr;
  t.dim_out = h->d_dimx + s + 1;
}

int run_gates(mps_state* h, const std::vector<GateRef>& gates) {
  if (gates.empty()) return MPS_OK;
  const bool dd = h->prec == MPS_PREC_DD;
  int capmax = 1;
  for (int b = 0; b <= h->n; ++b) capmax = std::max(capmax, h->capx[b]);
  int n2 = 0, n3 = 0;
  for (const auto& g : gates) {
    n2 += g.k == 2;
    n3 += g.k == 3;
  }
  const int Mcap = 2 * capmax, Ncap = (n3 ? 4 : 2) * capmax;
  const int t1cap = n3 ? 4 * capmax * capmax : 0;
  const int S = std::max(n3 ? 2 : 1,
                         std::min(std::min(h->max_slots, std::max(2, h->n / 2 + 1)), std::max(1, n2 + 2 * n3)));
  SchedBufs L;
  L.S = S;
  L.slot_bytes = slot_workspace_bytes(h, Mcap, Ncap, t1cap);
  int rc = ensure_ws(h, L.slot_bytes * S);
  if (rc) return rc;
  L.o_tasks = 0;
  L.o_flags = align_up(sizeof(Task2) * S);
  L.o_stats = L.o_flags + align_up(sizeof(int) * 3 * S);
  L.o_fro = L.o_stats + align_up(sizeof(double) * 8 * S);
  L.o_dims = L.o_fro + align_up(sizeof(double) * S);
  L.o_u8 = L.o_dims + align_up(sizeof(int) * (h->n + 1));
  L.o_ents = L.o_u8 + align_up(sizeof(double2) * 128 * S);
  const size_t list_bytes = align_up(std::max(sizeof(mpsk::Ent) * S, sizeof(Task1) * (size_t)h->n));
  L.o_end = L.o_ents + SchedBufs::kLists * list_bytes;
  rc = ensure_small(h, L.o_end);
  if (rc) return rc;
  Task2* ht = (Task2*)(h->h_stage + L.o_tasks);
  Task2* dt = (Task2*)(h->d_small + L.o_tasks);
  int* d_flags = (int*)(h->d_small + L.o_flags);
  int* hflags = (int*)(h->h_stage + L.o_flags);
  double* d_stats = (double*)(h->d_small + L.o_stats);
  double* hstats = (double*)(h->h_stage + L.o_stats);
  double* d_fro = (double*)(h->d_small + L.o_fro);
  double2* hu8 = (double2*)(h->h_stage + L.o_u8);
  double2* du8 = (double2*)(h->d_small + L.o_u8);
  enum { LN2 = 0, LN3, LJ, LD, LENTER, LFIN, LFIN3, LMID, LG1 };
  auto hlist = [&](int i) { return h->h_stage + L.o_ents + i * list_bytes; };
  auto dlist = [&](int i) { return h->d_small + L.o_ents + i * list_bytes; };

  std::vector<Slot> slot(S);
  std::vector<char> done(gates.size(), 0), busy(h->n, 0);
  std::vector<double> gstats(8 * gates.size(), 0.0);
  std::vector<int> gsweeps(gates.size(), 0), gdd(gates.size(), 0);
  size_t first_pending = 0;
  int status = MPS_OK;
  const int bw = h->block_width;
  const size_t window = (size_t)4 * S + 16;
  hipError_t e;

  auto upload_list = [&](int li, const std::vector<mpsk::Ent>& ents) -> mpsk::Ent* {
    mpsk::Ent* hl = (mpsk::Ent*)hlist(li);
    for (size_t i = 0; i < ents.size(); ++i) hl[i] = ents[i];
    hipError_t ee = hipMemcpyAsync(dlist(li), hl, sizeof(mpsk::Ent) * ents.size(), hipMemcpyHostToDevice, h->stream);
    return ee == hipSuccess ? (mpsk::Ent*)dlist(li) : nullptr;
  };
  auto ents_of = [&](const std::vector<int>& sl) {
    std::vector<mpsk::Ent> v;
    for (int si : sl) v.push_back(mpsk::Ent{si, slot[si].sweep});
    return v;
  };
  auto free_slot = [&]() {
    for (int si = 0; si < S; ++si)
      if (slot[si].state == 0) return si;
    return -1;
  };

  bool unsynced = false;  // async copies from the pinned staging may still be pending
  while (true) {
    // the staging buffers are rewritten below: wait for copies a previous tick left
    if (unsynced) {
      HIPCHK(h, hipStreamSynchronize(h->stream));
      unsynced = false;
    }
    // ---- 1. admission
    std::vector<int> new2, new3;
    std::vector<GateRef> g1;
    std::vector<char> claimed(h->n, 0);
    int free_slots = 0;
    for (auto& sl : slot) free_slots += sl.state == 0;
    while (first_pending < gates.size() && done[first_pending]) ++first_pending;
    for (size_t gi = first_pending; gi < gates.size() && gi < first_pending + window; ++gi) {
      if (done[gi]) continue;
      const GateRef& g = gates[gi];
      bool free_ = true;
      for (int q = g.first; q < g.first + g.k; ++q) free_ &= !busy[q] && !claimed[q];
      if (free_ && g.k == 1) {
        g1.push_back(g);
        done[gi] = 1;
        claimed[g.first] = 1;  // later gates on this site wait for the next pass
        continue;
      }
      if (free_ && ((g.k == 2 && free_slots >= 1) || (g.k == 3 && free_slots >= 2))) {
        const int si = free_slot();
        Slot& sl = slot[si];
        sl = Slot{};
        sl.state = 1;
        sl.gate = (int)gi;
        const int s0 = g.first;
        Task2& t = ht[si];
        if (g.k == 2) {
          setup_split(h, t, s0, h->dimx[s0], h->dimx[s0 + 1], h->dimx[s0 + 2]);
          for (int q = 0; q < 16; ++q) {
            t.U[q] = make_double2(g.U[2 * q], g.U[2 * q + 1]);
            t.U_lo[q] = (dd && g.Ulo) ? make_double2(g.Ulo[2 * q], g.Ulo[2 * q + 1]) : make_double2(0, 0);
          }
          new2.push_back(si);
        } else {
          setup_split(h, t, s0, h->dimx[s0], h->dimx[s0 + 1], h->dimx[s0 + 2]);
          t.B3 = h->B[s0 + 2];
          t.B3_lo = dd ? h->Blo[s0 + 2] : nullptr;
          t.ld3 = h->capx[s0 + 3];
          t.d = h->dimx[s0 + 3];
          t.N = 4 * t.d;
          double2* u8h = hu8 + 128 * si;
          for (int q = 0; q < 64; ++q) {
            u8h[q] = make_double2(g.U[2 * q], g.U[2 * q + 1]);
            u8h[64 + q] = (dd && g.Ulo) ? make_double2(g.Ulo[2 * q], g.Ulo[2 * q + 1]) : make_double2(0, 0);
          }
          t.U8 = du8 + 128 * si;
          t.U8_lo = du8 + 128 * si + 64;
          sl.kind = 1;
          const int sb = [&] {
            for (int j = 0; j < S; ++j)
              if (j != si && slot[j].state == 0) return j;
            return -1;
          }();
          slot[sb] = Slot{};
          slot[sb].state = 5;
          slot[sb].kind = 2;
          slot[sb].gate = (int)gi;
          sl.partner = sb;
          --free_slots;
          new3.push_back(si);
        }
        carve(h, t, h->ws + L.slot_bytes * si, d_flags, d_stats, d_fro, si);
        sl.M = t.M;
        sl.N = t.N;
        for (int q = g.first; q < g.first + g.k; ++q) busy[q] = 1;
        done[gi] = 1;
        --free_slots;
        continue;
      }
      for (int q = g.first; q < g.first + g.k; ++q) claimed[q] = 1;
    }
    if (!g1.empty()) {
      Task1* h1 = (Task1*)hlist(LG1);
      long maxel = 0;
      for (size_t i = 0; i < g1.size(); ++i) {
        const int s0 = g1[i].first;
        Task1 t{};
        t.B = h->B[s0];
        t.B_lo = dd ? h->Blo[s0] : nullptr;
        t.ld = h->capx[s0 + 1];
        t.a = h->dimx[s0];
        t.b = h->dimx[s0 + 1];
        for (int q = 0; q < 4; ++q) {
          t.U[q] = make_double2(g1[i].U[2 * q], g1[i].U[2 * q + 1]);
          t.U_lo[q] = (dd && g1[i].Ulo) ? make_double2(g1[i].Ulo[2 * q], g1[i].Ulo[2 * q + 1]) : make_double2(0, 0);
        }
        h1[i] = t;
        maxel = std::max(maxel, (long)t.a * t.b);
      }
      HIPCHK(h, hipMemcpyAsync(dlist(LG1), h1, sizeof(Task1) * g1.size(), hipMemcpyHostToDevice, h->stream));
      unsynced = true;
      Timed tm(h, 4);
      e = dd ? mpsk::launch_gate1_dd((Task1*)dlist(LG1), (int)g1.size(), maxel, h->stream)
             : mpsk::launch_gate1((Task1*)dlist(LG1), (int)g1.size(), maxel, h->stream);
      if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("gate1: ") + hipGetErrorString(e));
    }
    if (!new2.empty() || !new3.empty()) {
      HIPCHK(h, hipMemcpyAsync(dt, ht, sizeof(Task2) * S, hipMemcpyHostToDevice, h->stream));
      if (!new3.empty())
        HIPCHK(h, hipMemcpyAsync(du8, hu8, sizeof(double2) * 128 * S, hipMemcpyHostToDevice, h->stream));
      unsynced = true;
      Timed tm(h, 0);
      for (int which = 0; which < 2; ++which) {
        const std::vector<int>& nl = which ? new3 : new2;
        if (nl.empty()) continue;
        mpsk::Ent* el = upload_list(which ? LN3 : LN2, ents_of(nl));
        if (!el) return fail(h, MPS_EDEVICE, "list upload failed");
        int mM = 0, mN = 0, mA = 0, mC = 0, mD = 0;
        for (int si : nl) {
          mM = std::max(mM, slot[si].M);
          mN = std::max(mN, slot[si].N);
          mA = std::max(mA, ht[si].a);
          mC = std::max(mC, ht[si].c);
          mD = std::max(mD, ht[si].d);
        }
        e = mpsk::launch_prep2(dt, el, (int)nl.size(), mN, h->stream);
        if (e == hipSuccess) {
          if (which)
            e = mpsk::launch_theta3(dt, el, (int)nl.size(), mA, mC, mD, dd, h->stream);
          else
            e = dd ? mpsk::launch_theta2_dd(dt, el, (int)nl.size(), mM, mN, h->stream)
                   : mpsk::launch_theta2(dt, el, (int)nl.size(), mM, mN, h->stream);
        }
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("theta: ") + hipGetErrorString(e));
      }
    }
    // ---- 2. one sweep for every iterating slot
    std::vector<int> jl, dl;
    for (int si = 0; si < S; ++si) {
      if (slot[si].state == 1) jl.push_back(si);
      if (slot[si].state == 2) dl.push_back(si);
    }
    if (jl.empty() && dl.empty()) {
      bool any_active = false;
      for (auto& sl : slot) any_active |= sl.state != 0;
      if (!any_active) {
        while (first_pending < gates.size() && done[first_pending]) ++first_pending;
        if (first_pending >= gates.size()) break;
        continue;  // only single-site gates were pending; admit the rest
      }
    }
    if (!jl.empty()) {
      mpsk::Ent* el = upload_list(LJ, ents_of(jl));
      if (!el) return fail(h, MPS_EDEVICE, "list upload failed");
      int mN = 0;
      for (int si : jl) mN = std::max(mN, slot[si].N);
      const int nb = (mN + bw - 1) / bw;
      const int nsteps = nb + (nb & 1) - 1;
      Timed tm(h, 1, nsteps);
      h->slot_sweeps += (long)jl.size();
      for (int stp = 0; stp < nsteps; ++stp) {
        long long* pc = (h->d_phase && stp == nsteps / 2) ? h->d_phase : nullptr;
        e = mpsk::launch_jacobi_step(dt, el, (int)jl.size(), mN, bw, stp, h->tol_mult, h->max_inner, h->stream, pc);
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("jacobi: ") + hipGetErrorString(e));
      }
    }
    if (!dl.empty()) {
      mpsk::Ent* el = upload_list(LD, ents_of(dl));
      if (!el) return fail(h, MPS_EDEVICE, "list upload failed");
      int mN = 0;
      for (int si : dl) mN = std::max(mN, slot[si].N);
      const int nb = (mN + 7) / 8;
      const int nsteps = nb + (nb & 1) - 1;
      Timed tm(h, 6, nsteps);
      h->slot_sweeps_dd += (long)dl.size();
      for (int stp = 0; stp < nsteps; ++stp) {
        e = mpsk::launch_jacobi_step_dd(dt, el, (int)dl.size(), mN, stp, h->tol_mult, h->max_inner, h->stream);
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("dd jacobi: ") + hipGetErrorString(e));
      }
    }
    // ---- 3. convergence
    if (!jl.empty() || !dl.empty()) {
      HIPCHK(h, hipMemcpyAsync(hflags, d_flags, sizeof(int) * 3 * S, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      unsynced = false;
      if (h->d_phase && !jl.empty()) {
        long long pc[5];
        HIPCHK(h, hipMemcpy(pc, h->d_phase, sizeof(pc), hipMemcpyDeviceToHost));
        // wall_clock64 runs at 100 MHz on gfx950
        std::fprintf(stderr, "[mps] step phases (us, %zu updates, N %d): gram %.1f inner %.1f update %.1f rot %lld\n",
                     jl.size(), slot[jl[0]].N, (pc[1] - pc[0]) * 0.01, (pc[2] - pc[1]) * 0.01, (pc[3] - pc[2]) * 0.01,
                     pc[4]);
      }
    }
    std::vector<int> enter;
    for (int si : jl) {
      Slot& sl = slot[si];
      const bool rot = hflags[3 * si + sl.sweep % 3] != 0;
      ++sl.sweep;
      if (!rot || sl.sweep >= h->max_sweeps) {
        sl.fp64_sweeps = sl.sweep;
        sl.fp64_conv = !rot;
        if (dd) {
          enter.push_back(si);
          sl.state = 2;
          sl.sweep = 0;
        } else {
          sl.conv = sl.fp64_conv;
          sl.state = 3;
        }
      }
    }
    for (int si : dl) {
      Slot& sl = slot[si];
      const bool rot = hflags[3 * si + sl.sweep % 3] != 0;
      ++sl.sweep;
      if (!rot || sl.sweep >= h->max_sweeps_dd) {
        sl.dd_sweeps = sl.sweep;
        sl.conv = !rot;
        sl.state = 3;
      }
    }
    if (!enter.empty()) {
      unsynced = true;
      mpsk::Ent* el = upload_list(LENTER, ents_of(enter));
      if (!el) return fail(h, MPS_EDEVICE, "list upload failed");
      int mM = 0, mN = 0;
      for (int si : enter) { mM = std::max(mM, slot[si].M); mN = std::max(mN, slot[si].N); }
      Timed tm(h, 6);
      e = mpsk::launch_dd_enter(dt, el, (int)enter.size(), mM, mN, h->stream);
      if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("dd enter: ") + hipGetErrorString(e));
    }
    // ---- 4. finalise converged slots
    std::vector<int> fl, fl2, fl3;
    for (int si = 0; si < S; ++si)
      if (slot[si].state == 3) {
        fl.push_back(si);
        (slot[si].kind == 1 ? fl3 : fl2).push_back(si);
      }
    if (!fl.empty()) {
      mpsk::Ent* el = upload_list(LFIN, ents_of(fl));
      if (!el) return fail(h, MPS_EDEVICE, "list upload failed");
      int mM = 0, mN = 0;
      for (int si : fl) { mM = std::max(mM, slot[si].M); mN = std::max(mN, slot[si].N); }
      {
        Timed tm(h, 2);
        e = dd ? mpsk::launch_truncate_dd(dt, el, (int)fl.size(), h->chi, h->eps, h->rank_floor_dd, h->stream)
               : mpsk::launch_truncate(dt, el, (int)fl.size(), h->chi, h->eps, h->rank_floor, h->stream);
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("truncate: ") + hipGetErrorString(e));
      }
      {
        Timed tm(h, 3);
        for (int which = 0; which < 2; ++which) {
          const std::vector<int>& ll = which ? fl3 : fl2;
          if (ll.empty()) continue;
          mpsk::Ent* e2 = which ? upload_list(LFIN3, ents_of(ll)) : upload_list(LMID, ents_of(ll));
          if (!e2) return fail(h, MPS_EDEVICE, "list upload failed");
          int lM = 0, lN = 0;
          for (int si : ll) { lM = std::max(lM, slot[si].M); lN = std::max(lN, slot[si].N); }
          const int maxK = std::min(h->chi, std::min(lM, lN));
          e = dd ? mpsk::launch_split_dd(dt, e2, (int)ll.size(), lM, lN, maxK, h->stream, which == 0)
                 : mpsk::launch_split(dt, e2, (int)ll.size(), lM, lN, maxK, h->stream, which == 0);
          if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("split: ") + hipGetErrorString(e));
        }
      }
      HIPCHK(h, hipMemcpyAsync(hstats, d_stats, sizeof(double) * 8 * S, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipMemcpyAsync(h->h_stage + L.o_dims, h->d_dimx, sizeof(int) * (h->n + 1), hipMemcpyDeviceToHost,
                               h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      unsynced = false;
      std::memcpy(h->dimx.data(), h->h_stage + L.o_dims, sizeof(int) * (h->n + 1));
      // first splits of three-site gates: the second split takes over in the reserved slot
      std::vector<mpsk::Ent> mids;
      std::vector<int> newB;
      int mN1 = 0, mK1 = 0, mNB = 0;
      for (int si : fl3) {
        Slot& sa = slot[si];
        const GateRef& g = gates[sa.gate];
        const int s0 = g.first, sb = sa.partner;
        Task2& tb = ht[sb];
        setup_split(h, tb, s0 + 1, h->dimx[s0 + 1], 0, h->dimx[s0 + 3]);
        carve(h, tb, h->ws + L.slot_bytes * sb, d_flags, d_stats, d_fro, sb);
        Slot& sbl = slot[sb];
        sbl.state = 1;
        sbl.sweep = 0;
        sbl.M = tb.M;
        sbl.N = tb.N;
        gsweeps[sa.gate] = sa.fp64_sweeps;
        gdd[sa.gate] = sa.dd_sweeps;
        if (!sa.conv) status = MPS_ENOCONV;
        mids.push_back(mpsk::Ent{si, sb});
        newB.push_back(sb);
        mN1 = std::max(mN1, sa.N);
        mK1 = std::max(mK1, std::min(h->chi, sa.M));
        mNB = std::max(mNB, tb.N);
      }
      if (!mids.empty()) {
        HIPCHK(h, hipMemcpyAsync(dt, ht, sizeof(Task2) * S, hipMemcpyHostToDevice, h->stream));
        unsynced = true;
        mpsk::Ent* eb = upload_list(LN2, ents_of(newB));
        mpsk::Ent* em = upload_list(LN3, mids);
        if (!eb || !em) return fail(h, MPS_EDEVICE, "list upload failed");
        Timed tm(h, 0);
        e = mpsk::launch_prep2(dt, eb, (int)newB.size(), mNB, h->stream);
        if (e == hipSuccess) e = mpsk::launch_mid3(dt, em, (int)mids.size(), mN1, mK1, dd, h->stream);
        if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("mid: ") + hipGetErrorString(e));
        for (int si : fl3) slot[si] = Slot{};  // its V is read by the mid kernel, queued before any reuse
      }
      for (int si : fl2) {
        Slot& sl = slot[si];
        const GateRef& g = gates[sl.gate];
        std::memcpy(&gstats[8 * sl.gate], hstats + 8 * si, sizeof(double) * 8);
        gsweeps[sl.gate] = std::max(gsweeps[sl.gate], sl.fp64_sweeps);
        gdd[sl.gate] = std::max(gdd[sl.gate], sl.dd_sweeps);
        if (!sl.conv) status = MPS_ENOCONV;
        if (h->debug_sweeps)
          std::fprintf(stderr, "[mps] update at site %d (M %d, N %d, kind %d): %d FP64 sweeps, %d dd sweeps\n",
                       g.first, sl.M, sl.N, sl.kind, sl.fp64_sweeps, sl.dd_sweeps);
        for (int q = g.first; q < g.first + g.k; ++q) busy[q] = 0;
        sl = Slot{};
      }
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  // diagnostics of the last multi-site gate in queue order
  h->last.splits = 0;
  for (size_t gi = gates.size(); gi-- > 0;) {
    if (gates[gi].k == 1) continue;
    const double* st = &gstats[8 * gi];
    h->last.W = st[0];
    h->last.w = st[1];
    h->last.gap = st[2];
    h->last.epsdist = st[3];
    h->last.k = (int)st[4];
    h->last.rank = (int)st[5];
    h->last.sweeps = *std::max_element(gsweeps.begin(), gsweeps.end());
    h->last.dd_sweeps = *std::max_element(gdd.begin(), gdd.end());
    h->last.splits = gates[gi].k - 1;
    break;
  }
  if (status) return fail(h, status, "Jacobi sweep limit reached");
  return MPS_OK;
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
  if (const char* dbg = std::getenv("MPS_DEBUG_SWEEPS")) h->debug_sweeps = dbg[0] == '1';
  if (const char* dbg = std::getenv("MPS_DEBUG_PHASES"))
    if (dbg[0] == '1' && hipMalloc((void**)&h->d_phase, 8 * sizeof(long long)) != hipSuccess) h->d_phase = nullptr;
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
  if (h->d_phase) (void)hipFree(h->d_phase);
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
  if (!h || cls < 0 || cls >= 10) return MPS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  harvest_timing(h);
  if (cls >= 8) {  // counters: update-sweeps of the FP64 Jacobi (8) and of the dd polish (9)
    long& c = cls == 8 ? h->slot_sweeps : h->slot_sweeps_dd;
    if (ms) *ms = 0.0;
    if (launches) *launches = c;
    if (reset) c = 0;
    return MPS_OK;
  }
  if (ms) *ms = h->tms[cls];
  if (launches) *launches = h->tcount[cls];
  if (reset) { h->tms[cls] = 0; h->tcount[cls] = 0; }
  return MPS_OK;
}

}  // extern "C"
