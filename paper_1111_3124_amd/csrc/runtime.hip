// Host runtime of the MPS gate-update library: engines (stream, workspace arena,
// staging, timing), states, the update scheduler and the C ABI of include/mps.h.
//
// An engine owns everything a run of the scheduler needs besides the states: one
// standalone handle owns one engine; a batch owns one engine shared by all its
// states, so the updates of every circuit of the batch run in the same launches.
// Bond dimensions live in device tables written by the truncation kernel; the
// host mirrors them after each finalisation (one small device-to-host copy), so
// that every launch is sized to the live shapes.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <deque>
#include <fstream>
#include <sstream>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mps.h"
#include "common.h"
#include "dd.h"
#include "dd_kernels.h"
#include "ddref.h"
#include "kernels3.h"
#include "launch.h"
#include "rdo.h"

using mpsk::Task1;
using mpsk::Task2;

namespace {

thread_local std::string g_create_error;

struct EvPair {
  hipEvent_t a, b;
  int cls;
  int n;
};

// First-fit allocator of offsets in the workspace arena, with coalescing.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> fr;  // offset -> length of each free block
  void reset(size_t s) {
    size = s;
    fr.clear();
    if (s) fr[0] = s;
  }
  size_t alloc(size_t len) {
    for (auto it = fr.begin(); it != fr.end(); ++it)
      if (it->second >= len) {
        const size_t off = it->first, rem = it->second - len;
        fr.erase(it);
        if (rem) fr[off + len] = rem;
        return off;
      }
    return SIZE_MAX;
  }
  void release(size_t off, size_t len) {
    auto it = fr.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != fr.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      fr.erase(nx);
    }
    if (it != fr.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        fr.erase(it);
      }
    }
  }
};

}  // namespace

// One row of a tuning table: the step kernel configuration of Jacobi problems with
// at most nmax columns at one precision, measured fastest on this device (written by
// the package's autotuner).
struct TuneEntry {
  int prec = 0, nmax = 0;
  int bw = 8, inner_few = 1, qr = 1;
};

struct Engine {
  int prec = MPS_PREC_FP64;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // the Jacobi steps of a tick run as two interleaved launch sequences (half the
  // iterating updates each) on stream and stream2, so that one half's memory phases
  // overlap the other half's inner Jacobi
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // QR factorisations of newly admitted updates run on stream3, overlapping the
  // tick's Jacobi sweep of the updates already iterating
  hipStream_t stream3 = nullptr;
  hipEvent_t ev_qr = nullptr;
  // dd refinement passes, dd polish sweeps and the dd promotion of converged updates
  // run on stream4, overlapping the FP64 sweeps of the others; joined before every
  // readback of the rotation flags
  hipStream_t stream4 = nullptr;
  hipEvent_t ev_dd_fork = nullptr, ev_dd_join = nullptr;
  bool dd_stream = true;
  int jacobi_streams = 2;
  bool fuse = true;  // mps_apply_gates multiplies single-site gates into neighbours
  bool qr = true;   // QR preconditioning of two-site Jacobi problems
  // block width 8: a step launch serving at most this many updates runs as two launches
  // of half-sized blocks (more blocks for few updates); 0: never
  int split_max = 4;
  int device = 0;
  bool batch = false;  // a batch engine sizes workspace per update, not per slot
  // options (shared by every state of the engine)
  int max_sweeps = 40;
  int max_sweeps_dd = 16;
  int max_inner = 1;
  // inner sweeps per block pair, tasks with fewer than 16 blocks: one for FP64 (the
  // cheapest overall); dd engines keep every pair diagonalised per step (12), the
  // starting point their refinement and polish expect on rank-deficient thetas
  int max_inner_few = 1;
  int block_width = 8;
  // per-size step configurations from the tuning table of this device (see
  // TuneEntry); off once block width, inner-sweep limit or QR is set explicitly
  bool tuned = true;
  std::vector<struct TuneEntry> tune;
  int max_slots = 32;
  double ws_limit = 16.0 * (1ull << 30);  // batch engines: workspace arena cap, bytes
  double tol_mult = 1.0;
  bool dd_refine = true;  // dd: simultaneous first-order corrections before any pairwise polish
  int max_ref_passes = 4;
  double rank_floor = 0x1p-44;
  double rank_floor_dd = 0x1p-96;
  bool timing = false;
  bool debug_sweeps = false;  // MPS_DEBUG_SWEEPS=1: print per-update sweep counts
  // workspace
  char* ws = nullptr;
  size_t ws_size = 0;
  Arena arena;
  char* h_stage = nullptr;  // pinned host staging (task arrays, readbacks)
  size_t h_stage_size = 0;
  char* d_small = nullptr;  // device task arrays + flags + stats
  size_t d_small_size = 0;
  // timing
  std::vector<EvPair> pending;
  std::vector<hipEvent_t> evpool;
  double tms[8] = {0};
  long tcount[8] = {0};
  long slot_sweeps = 0, slot_sweeps_dd = 0;  // update-sweeps executed (FP64, dd polish)
  long noconv_updates = 0;                    // splits finalised at a sweep limit
  long long* d_phase = nullptr;               // MPS_DEBUG_PHASES=1: step phase stamps
  // Jacobi sweeps per tick (1 or 2) and whether they are replayed from captured graphs
  int tick_sweeps = 2;
  bool graphs_on = false;
  std::map<std::vector<long long>, hipGraphExec_t> graphs;
  long graphs_built = 0, graph_launches = 0;
};

struct mps_state {
  int n = 0, chi = 0, prec = MPS_PREC_FP64;
  double eps = 0.0;
  Engine* E = nullptr;
  bool own_engine = false;
  mps_batch* batch = nullptr;  // non-null: a member of a batch (which owns its memory)
  char* mem = nullptr;         // device block holding B, B_lo, V, V_lo, dims (standalone)
  std::vector<int> capx;  // capx[b+1] = capacity of bond b; capx[0] = capx[n] = 1
  std::vector<int> dimx;  // host mirror of the bond dims, same indexing
  int* d_dimx = nullptr;
  std::vector<double2*> B, Blo;  // per site, capx[s] * 2 * capx[s+1]
  double* d_lam = nullptr;       // (n+1) slots x chi; slot b+1 = bond b; slots 0, n = [1]
  double* d_lam_lo = nullptr;
  mps_update_stats last{};
  std::string err;
  // room for any message this library writes, so that an error on a path that must
  // not allocate (mps_amplitudes_noalloc) does not grow the string
  mps_state() { err.reserve(256); }
};

struct mps_batch {
  Engine* E = nullptr;
  std::vector<mps_state*> units;
  char* mem = nullptr;  // one device block for every state
  int* d_dims = nullptr;  // all bond-dimension tables, back to back
  int dims_total = 0;
  std::string err;
};

namespace {

int fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}
int fail(mps_state* h, int code, const std::string& msg) { return fail(h ? &h->err : nullptr, code, msg); }
int fail(mps_batch* b, int code, const std::string& msg) { return fail(b ? &b->err : nullptr, code, msg); }

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
constexpr int kQrMaxN = 1024;

// ------------------------------------------------------------------ tuning table
// A text file of sections
//     key <arch> <hip runtime version>
//     <fp64|dd> <nmax> <block width> <inner sweeps, few blocks> <qr 0|1>
// (lines starting with # are comments).  The section whose key matches the device
// and the runtime is used; without one the built-in defaults apply.  The file is
// $MPS_TUNING_FILE, else tuning.txt beside this library.
std::string tuning_key(int device) {
  hipDeviceProp_t prop;
  int ver = 0;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess || hipRuntimeGetVersion(&ver) != hipSuccess) return "";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + " " + std::to_string(ver);
}

std::string tuning_path() {
  if (const char* p = std::getenv("MPS_TUNING_FILE")) return p;
  Dl_info info;
  if (dladdr((void*)&tuning_path, &info) && info.dli_fname) {
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning.txt";
  }
  return "tuning.txt";
}

std::vector<TuneEntry> load_tuning(const std::string& key) {
  std::vector<TuneEntry> out;
  std::ifstream f(tuning_path());
  if (!f || key.empty()) return out;
  std::string line;
  bool in = false;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string w;
    if (!(ls >> w) || w[0] == '#') continue;
    if (w == "key") {
      std::string arch, ver;
      ls >> arch >> ver;
      in = (arch + " " + ver) == key;
      continue;
    }
    if (!in || (w != "fp64" && w != "dd")) continue;
    TuneEntry t;
    t.prec = w == "dd" ? MPS_PREC_DD : MPS_PREC_FP64;
    if (!(ls >> t.nmax >> t.bw >> t.inner_few >> t.qr)) continue;
    if ((t.bw != 4 && t.bw != 8 && t.bw != 16) || t.inner_few < 1 || t.inner_few > 64 || t.nmax < 1) continue;
    out.push_back(t);
  }
  std::sort(out.begin(), out.end(), [](const TuneEntry& a, const TuneEntry& b) {
    return a.prec != b.prec ? a.prec < b.prec : a.nmax < b.nmax;
  });
  return out;
}

// the tables read so far, by key (each file is read once per key and process)
std::mutex g_tune_mu;
std::map<std::string, std::vector<TuneEntry>> g_tune;

std::vector<TuneEntry> tuning_for(int device) {
  const std::string key = tuning_key(device);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) it = g_tune.emplace(key, load_tuning(key)).first;
  return it->second;
}

// step configuration of a Jacobi problem with N columns: the first table row of the
// engine's precision with N <= nmax, else the engine's options
struct StepCfg {
  int bw, inner_few, qr;
};
StepCfg step_cfg(const Engine* E, int N) {
  if (E->tuned)
    for (const TuneEntry& t : E->tune)
      if (t.prec == E->prec && N <= t.nmax) return StepCfg{t.bw, t.inner_few, t.qr};
  return StepCfg{E->block_width, E->max_inner_few, E->qr ? 1 : 0};
}

// ------------------------------------------------------------------ engines
void engine_free(Engine* E);

Engine* engine_new(int prec, void* hip_stream, std::string* err) {
  Engine* E = new Engine();
  E->prec = prec;
  if (prec == MPS_PREC_DD) E->max_inner_few = 12;
  if (const char* dbg = std::getenv("MPS_DEBUG_SWEEPS")) E->debug_sweeps = dbg[0] == '1';
  hipError_t e = hipGetDevice(&E->device);
  if (e == hipSuccess) {
    if (hip_stream) {
      E->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking);
      E->own_stream = e == hipSuccess;
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream3, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev_qr, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->stream4, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev_dd_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&E->ev_dd_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    *err = std::string("engine: ") + hipGetErrorString(e);
    engine_free(E);
    return nullptr;
  }
  if (e == hipSuccess) E->tune = tuning_for(E->device);
  if (const char* dbg = std::getenv("MPS_DEBUG_PHASES"))
    if (dbg[0] == '1' && hipMalloc((void**)&E->d_phase, 8 * sizeof(long long)) != hipSuccess) E->d_phase = nullptr;
  return E;
}

// wait for every stream of the engine (before memory that kernels may touch is freed)
void engine_sync(Engine* E) {
  if (!E) return;
  for (hipStream_t q : {E->stream, E->stream2, E->stream3, E->stream4})
    if (q) (void)hipStreamSynchronize(q);
}

void engine_free(Engine* E) {
  if (!E) return;
  if (E->stream) (void)hipStreamSynchronize(E->stream);
  if (E->stream2) {
    (void)hipStreamSynchronize(E->stream2);
    (void)hipStreamDestroy(E->stream2);
  }
  if (E->stream3) {
    (void)hipStreamSynchronize(E->stream3);
    (void)hipStreamDestroy(E->stream3);
  }
  if (E->stream4) {
    (void)hipStreamSynchronize(E->stream4);
    (void)hipStreamDestroy(E->stream4);
  }
  if (E->ev_dd_fork) (void)hipEventDestroy(E->ev_dd_fork);
  if (E->ev_dd_join) (void)hipEventDestroy(E->ev_dd_join);
  if (E->ev_qr) (void)hipEventDestroy(E->ev_qr);
  if (E->ev_fork) (void)hipEventDestroy(E->ev_fork);
  if (E->ev_join) (void)hipEventDestroy(E->ev_join);
  for (auto& kv : E->graphs) (void)hipGraphExecDestroy(kv.second);
  E->graphs.clear();
  if (E->d_phase) (void)hipFree(E->d_phase);
  if (E->ws) (void)hipFree(E->ws);
  if (E->d_small) (void)hipFree(E->d_small);
  if (E->h_stage) (void)hipHostFree(E->h_stage);
  for (auto& p : E->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : E->evpool) (void)hipEventDestroy(e);
  if (E->own_stream && E->stream) (void)hipStreamDestroy(E->stream);
  delete E;
}

hipEvent_t ev_get(Engine* E) {
  if (!E->evpool.empty()) {
    hipEvent_t e = E->evpool.back();
    E->evpool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct Timed {
  Engine* E;
  EvPair p{};
  bool on;
  hipStream_t s;
  // `launches` kernels are enqueued on stream `ss` (default: the engine's) between
  // the two events
  Timed(Engine* EE, int cls, int launches = 1, hipStream_t ss = nullptr)
      : E(EE), on(EE->timing), s(ss ? ss : EE->stream) {
    if (on) {
      p.a = ev_get(E);
      p.b = ev_get(E);
      p.cls = cls;
      p.n = launches;
      (void)hipEventRecord(p.a, s);
    }
  }
  ~Timed() {
    if (on) {
      (void)hipEventRecord(p.b, s);
      E->pending.push_back(p);
    }
  }
};

// after a synchronisation: fold finished event pairs into the per-class totals
void harvest_timing(Engine* E) {
  for (auto& p : E->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      E->tms[p.cls] += ms;
      E->tcount[p.cls] += p.n;
    }
    E->evpool.push_back(p.a);
    E->evpool.push_back(p.b);
  }
  E->pending.clear();
}

// the arena must hold `bytes`; only called while no update holds workspace
int ensure_ws(Engine* E, size_t bytes, std::string* err) {
  if (bytes > E->ws_size) {
    HIPCHK(err, hipStreamSynchronize(E->stream));
    HIPCHK(err, hipStreamSynchronize(E->stream4));
    if (E->ws) HIPCHK(err, hipFree(E->ws));
    E->ws = nullptr;
    E->ws_size = 0;
    HIPCHK(err, hipMalloc((void**)&E->ws, bytes));
    E->ws_size = bytes;
  }
  E->arena.reset(E->ws_size);
  return MPS_OK;
}

int ensure_small(Engine* E, size_t bytes, std::string* err) {
  if (bytes <= E->d_small_size && bytes <= E->h_stage_size) return MPS_OK;
  HIPCHK(err, hipStreamSynchronize(E->stream));
  size_t want = std::max<size_t>(bytes, 1 << 16);
  if (bytes > E->d_small_size) {
    if (E->d_small) HIPCHK(err, hipFree(E->d_small));
    E->d_small = nullptr;
    HIPCHK(err, hipMalloc((void**)&E->d_small, want));
    E->d_small_size = want;
  }
  if (bytes > E->h_stage_size) {
    if (E->h_stage) HIPCHK(err, hipHostFree(E->h_stage));
    E->h_stage = nullptr;
    HIPCHK(err, hipHostMalloc((void**)&E->h_stage, want, hipHostMallocDefault));
    E->h_stage_size = want;
  }
  return MPS_OK;
}

// ------------------------------------------------------------------ state memory
// One device block per state: site tensors (hi planes, then lo planes), Schmidt
// value slots (hi, lo) and the bond-dimension table.
void state_shape(mps_state* h, int n, int chi, double eps, int prec) {
  h->n = n;
  h->chi = chi;
  h->eps = eps;
  h->prec = prec;
  h->capx.assign(n + 1, 1);
  for (int b = 0; b + 1 < n; ++b) h->capx[b + 1] = bond_capacity(n, chi, b);
  h->dimx.assign(n + 1, 1);
}

size_t state_bytes(const mps_state* h, bool with_dims) {
  const bool dd = h->prec == MPS_PREC_DD;
  size_t b = 0;
  for (int s = 0; s < h->n; ++s) b += align_up((size_t)h->capx[s] * 2 * h->capx[s + 1] * sizeof(double2)) * (dd ? 2 : 1);
  b += align_up((size_t)(h->n + 1) * h->chi * sizeof(double)) * (dd ? 2 : 1);
  if (with_dims) b += align_up(sizeof(int) * (h->n + 1));
  return b;
}

// carve the pointers of h from `base`; returns the end
char* state_carve(mps_state* h, char* base, bool with_dims) {
  const bool dd = h->prec == MPS_PREC_DD;
  h->B.assign(h->n, nullptr);
  h->Blo.assign(dd ? h->n : 0, nullptr);
  for (int plane = 0; plane < (dd ? 2 : 1); ++plane)
    for (int s = 0; s < h->n; ++s) {
      (plane ? h->Blo : h->B)[s] = (double2*)base;
      base += align_up((size_t)h->capx[s] * 2 * h->capx[s + 1] * sizeof(double2));
    }
  const size_t lam_b = align_up((size_t)(h->n + 1) * h->chi * sizeof(double));
  h->d_lam = (double*)base;
  base += lam_b;
  if (dd) {
    h->d_lam_lo = (double*)base;
    base += lam_b;
  }
  if (with_dims) {
    h->d_dimx = (int*)base;
    base += align_up(sizeof(int) * (h->n + 1));
  }
  return base;
}

// |0...0> for every state on zeroed memory: B_s[0][0][0] = 1, first value of each
// Schmidt slot = 1, all bond dims 1
int set_product_states(Engine* E, const std::vector<mps_state*>& hs, int* dims, long n_dims, std::string* err) {
  std::vector<double*> ones;
  for (mps_state* h : hs) {
    for (int s = 0; s < h->n; ++s) ones.push_back((double*)h->B[s]);
    for (int sl = 0; sl <= h->n; ++sl) ones.push_back(h->d_lam + (size_t)sl * h->chi);
  }
  double** d_ones = nullptr;
  HIPCHK(err, hipMalloc((void**)&d_ones, sizeof(double*) * ones.size()));
  hipError_t e = hipMemcpy(d_ones, ones.data(), sizeof(double*) * ones.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = mpsk::launch_set_product(d_ones, (long)ones.size(), dims, n_dims, E->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(E->stream);
  (void)hipFree(d_ones);
  if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("state set-up: ") + hipGetErrorString(e));
  for (mps_state* h : hs) h->dimx.assign(h->n + 1, 1);
  return MPS_OK;
}

bool finite_gate(int k, const double* U) {
  const int nd = 2 << (2 * k);
  for (int i = 0; i < nd; ++i)
    if (!std::isfinite(U[i])) return false;
  return true;
}

int validate_gate(const mps_state* h, int first, int k, const double* U, const double* Ulo, std::string* err) {
  if (k < 1 || k > 3) return fail(err, MPS_EINVAL, "k must be 1, 2 or 3");
  if (first < 0 || first + k > h->n) return fail(err, MPS_EINVAL, "gate sites out of range");
  if (!U) return fail(err, MPS_EINVAL, "null gate matrix");
  if (!finite_gate(k, U) || (Ulo && !finite_gate(k, Ulo)))
    return fail(err, MPS_ENONFINITE, "gate matrix has a NaN or infinite entry");
  return MPS_OK;
}

struct GateRef {
  int unit;  // index of the state in the run's state list
  int first, k;
  const double* U;
  const double* Ulo;
};

// ------------------------------------------------------------------ update scheduler
// Continuous batching of gate updates over one or more states.  Each two-site
// split occupies a slot (task descriptor + workspace from the engine's arena).
// One scheduler tick:
//   1. admit queued gates whose sites are free and not claimed by an earlier queued
//      gate of the same state (gates on disjoint sites commute, so queue order is
//      kept where it matters; states are independent): a single-site gate runs at
//      once; a two-site gate takes a slot and gets its prep + theta launch; a
//      three-site gate takes a slot for its first split (s | s+1 s+2) and reserves
//      a second one for its second split;
//   2. one Jacobi sweep for every slot still iterating (FP64 sweeps, or dd polish
//      sweeps after the FP64 iteration of a dd state has converged);
//   3. read the rotation flags; converged slots are truncated and split at once and
//      their new bond dimensions read back.  A finished first split of a three-site
//      gate hands Z1_k^H, weighted by its new Schmidt values, to the reserved slot as
//      the theta of the second split; any other finished slot frees its sites.
// A slow update never holds back updates that do not depend on it.
struct Slot {
  int state = 0;  // 0 free, 1 FP64 Jacobi, 2 dd refinement passes, 4 dd pairwise polish,
                  // 3 ready to finalise, 5 reserved
  int kind = 0;   // 0 two-site, 1 three-site first split, 2 three-site second split
  int gate = -1;
  int partner = -1;  // kind 1: the reserved slot of the second split
  int sweep = 0;
  int fp64_sweeps = 0, dd_sweeps = 0;
  bool fp64_conv = false, conv = false;
  int M = 0, Nt = 0, JM = 0, N = 0;  // theta rows and columns, Jacobi rows and columns
  int bw = 8, inner_few = 1;          // step kernel configuration (step_cfg)
  size_t ws_off = 0, ws_len = 0;  // workspace held in the arena
};

// Workspace of a task with an M x Nt theta: theta and theta_w (later W; for a wide
// theta theta_w^H, then Z), V (N x N, N = min(M, Nt)), the dd scratch (two N x N, one
// M x N), sigma^2, the order and T1 (three-site first split).
// partial Grams of the split Jacobi step (block width 8): the pairs of the padded
// block count, two row halves, two 16 x 16 parts
size_t jg_doubles(int N) { return (size_t)((N + 7) / 8 + 2) / 2 * 2 * 2 * 256; }

size_t task_ws_bytes(bool dd, int M, int Nt, int t1) {
  const int N = std::min(M, Nt), P = dd ? 2 : 1;
  const size_t MN = (size_t)M * Nt, NN = (size_t)N * N;
  size_t b = align_up((2 * MN + NN) * sizeof(double2)) * P;
  if (dd) b += 2 * align_up(NN * sizeof(double2)) + align_up(MN * sizeof(double2));
  b += align_up(N * sizeof(double)) * P + align_up(N * sizeof(int));
  b += align_up((size_t)t1 * sizeof(double2)) * P;
  // QR preconditioning: order, reflector heads, scales, panel factors (16 x 16 each)
  b += align_up(N * sizeof(int)) + align_up(N * sizeof(double2)) + align_up(N * sizeof(double)) +
       align_up((size_t)((N + 15) / 16) * 256 * sizeof(double2));
  b += align_up(jg_doubles(N) * sizeof(double));  // split Jacobi step: partial Grams
  return b;
}

// a bound over every task with M <= Mcap and Nt <= Ncap (task_ws_bytes is monotone)
size_t task_ws_bound(bool dd, int Mcap, int Ncap, int t1) { return task_ws_bytes(dd, Mcap, Ncap, t1); }

// theta columns; a wide theta (Nt > M) runs its one-sided Jacobi on theta_w^H, whose
// M columns are independent (theta_w's Nt columns would have to be driven to rank M)
void set_cols(Task2& t, int Nt) {
  t.Nt = Nt;
  t.tr = Nt > t.M ? 1 : 0;
  t.JM = t.tr ? Nt : t.M;
  t.N = t.tr ? t.M : Nt;
}

// workspace pointers of a task (shape already set), carved from the region w
void carve(bool dd, Task2& t, char* w, int* d_flags, double* d_stats, double* d_fro, int slot) {
  const size_t MN = (size_t)t.M * t.Nt, NN = (size_t)t.N * t.N;
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
    t.aux3 = (double2*)w;
    w += align_up(MN * sizeof(double2));
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
    if (dd) {
      t.T1_lo = (double2*)w;
      w += align_up(t1 * sizeof(double2));
    }
  }
  t.qperm = (int*)w;
  w += align_up(t.N * sizeof(int));
  t.qvd = (double2*)w;
  w += align_up(t.N * sizeof(double2));
  t.qt = (double*)w;
  w += align_up(t.N * sizeof(double));
  t.qT = (double2*)w;
  w += align_up((size_t)((t.N + 15) / 16) * 256 * sizeof(double2));
  t.JG = (double*)w;
  w += align_up(jg_doubles(t.N) * sizeof(double));
  t.qr = 0;
  t.JW = t.thw;
  t.JV = t.V;
  t.JR = t.JM;
  t.jvec = 1;
  // the split's right factor: V, or for a wide theta W itself (its kept columns are
  // scaled to unit norm after the truncation)
  t.Z = t.tr ? t.thw : t.V;
  t.Z_lo = t.tr ? t.thw_lo : t.V_lo;
  t.flags = d_flags + 3 * slot;
  t.stats = d_stats + 8 * slot;
  t.fro2 = d_fro + slot;
}

// QR preconditioning of a two-site task (theta_w P = Q R, Jacobi on R^H): tall or
// square thetas with 64 <= N and M <= 1024 (the panel kernel keeps at most two rows
// a thread), and for double-double only square ones (their refinement then runs on
// the transposed problem from the left singular vectors Q V).  FP64: the Jacobi's W
// is R^H in V's storage, V is not accumulated, Z is formed in theta_w's storage.
void qr_select(bool dd, Task2& t) {
  if (t.tr || t.N < 64 || t.M > 1024 || t.N > kQrMaxN || (dd && t.M != t.N)) return;
  t.qr = 1;
  t.JR = t.N;
  if (dd) {
    t.JW = t.aux1;
    t.JV = t.V;
    t.jvec = 1;
  } else {
    t.JW = t.V;
    t.JV = nullptr;
    t.jvec = 0;
    t.Z = t.thw;
  }
}

// a QR-preconditioned dd task after its FP64 Jacobi (V = Q V_x, the left singular
// vectors): from here on it is refined as the transposed problem theta_w^H V = W
void qr_to_transposed(Task2& t) {
  t.qr = 0;
  t.tr = 1;
  t.JM = t.Nt;
  t.N = t.M;
  t.Z = t.thw;
  t.Z_lo = t.thw_lo;
  t.JW = t.thw;
  t.JV = t.V;
  t.JR = t.JM;
  t.jvec = 1;
}

// the two-site split of state h between sites s and s+1 with bond dims a | (b) | c
void setup_split(const mps_state* h, Task2& t, int s, int a, int b, int c) {
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
  set_cols(t, 2 * c);
  t.lamL = h->d_lam + (size_t)s * h->chi;
  t.lamL_lo = dd ? h->d_lam_lo + (size_t)s * h->chi : nullptr;
  t.lamS = h->d_lam + (size_t)(s + 1) * h->chi;
  t.lamS_lo = dd ? h->d_lam_lo + (size_t)(s + 1) * h->chi : nullptr;
  t.dim_out = h->d_dimx + s + 1;
  t.chi = h->chi;
  t.eps = h->eps;
}

// workspace of a gate's tasks (upper bound over the live dims: capacities)
size_t gate_need_cap(bool dd, const mps_state* h, int first, int k) {
  if (k == 2) return task_ws_bound(dd, 2 * h->capx[first], 2 * h->capx[first + 2], 0);
  if (k == 3)
    return task_ws_bound(dd, 2 * h->capx[first], 4 * h->capx[first + 3], 4 * h->capx[first] * h->capx[first + 2]) +
           task_ws_bound(dd, 2 * h->capx[first + 1], 2 * h->capx[first + 3], 0);
  return 0;
}

// ------------------------------------------------------------------ Jacobi sweeps
// The FP64 Jacobi sweeps of one tick.  The iterating updates form groups that share
// a step kernel configuration (block width, inner-sweep limit); each group's updates
// are split into two halves, whose step launches run on the engine's stream and on
// stream2.  One sweep = the column-order kernel for every update, then the steps of
// the round-robin schedule.  An update whose previous sweep rotated nothing leaves
// each of its blocks at once (the kernels read its rotation flags), so sweeps past
// its convergence change nothing: a tick may run K sweeps and read the flags once.
struct SweepGroup {
  int bw = 8, inner_few = 1;
  int na = 0, nb = 0;  // updates of the two halves
  int oa = 0, ob = 0;  // their offsets in the sweep's half lists
  int mNa = 0, mNb = 0;
  bool split_a = false, split_b = false;
};

struct SweepPlan {
  std::vector<SweepGroup> groups;
  int n_order = 0;  // updates in the order list
  bool two = false;
  int K = 1;        // sweeps
  mpsk::Ent* la[2] = {nullptr, nullptr};  // per sweep: half-a list, half-b list, order list
  mpsk::Ent* lb[2] = {nullptr, nullptr};
  mpsk::Ent* lo[2] = {nullptr, nullptr};
  long long* phase = nullptr;  // debug stamps of one step (direct launches only)
};

int steps_of(int N, int bw) {
  const int nb = (N + bw - 1) / bw;
  return nb + (nb & 1) - 1;
}

int plan_steps(const SweepPlan& P) {
  int m = 0;
  for (const SweepGroup& g : P.groups) m = std::max(m, std::max(steps_of(g.mNa, g.bw), g.nb ? steps_of(g.mNb, g.bw) : 0));
  return m;
}

// enqueue the plan's K sweeps on st (and stream2): also the body of a captured graph
hipError_t enqueue_sweeps(Engine* E, Task2* dt, const SweepPlan& P, hipStream_t st) {
  hipError_t e = hipSuccess;
  const int nsteps = plan_steps(P);
  for (int k = 0; k < P.K; ++k) {
    e = mpsk::launch_jacobi_order(dt, P.lo[k], P.n_order, st);
    if (e != hipSuccess) return e;
    if (P.two) {
      if ((e = hipEventRecord(E->ev_fork, st)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(E->stream2, E->ev_fork, 0)) != hipSuccess) return e;
    }
    for (int stp = 0; stp < nsteps; ++stp) {
      for (const SweepGroup& g : P.groups) {
        long long* pc = (P.phase && k == 0 && stp == nsteps / 2 && &g == &P.groups[0]) ? P.phase : nullptr;
        if (g.na && stp < steps_of(g.mNa, g.bw)) {
          e = (g.split_a && !pc)
                  ? mpsk::launch_jacobi_split(dt, P.la[k] + g.oa, g.na, g.mNa, stp, E->tol_mult, E->max_inner,
                                              g.inner_few, st)
                  : mpsk::launch_jacobi_step(dt, P.la[k] + g.oa, g.na, g.mNa, g.bw, stp, E->tol_mult, E->max_inner,
                                             g.inner_few, st, pc);
          if (e != hipSuccess) return e;
        }
        if (g.nb && stp < steps_of(g.mNb, g.bw)) {
          hipStream_t s2 = P.two ? E->stream2 : st;
          e = g.split_b ? mpsk::launch_jacobi_split(dt, P.lb[k] + g.ob, g.nb, g.mNb, stp, E->tol_mult, E->max_inner,
                                                    g.inner_few, s2)
                        : mpsk::launch_jacobi_step(dt, P.lb[k] + g.ob, g.nb, g.mNb, g.bw, stp, E->tol_mult,
                                                   E->max_inner, g.inner_few, s2, nullptr);
          if (e != hipSuccess) return e;
        }
      }
    }
    if (P.two) {
      if ((e = hipEventRecord(E->ev_join, E->stream2)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st, E->ev_join, 0)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// the plan's launch sequence as an instantiated graph (captured on first use and
// kept while the engine lives); its shape and every device address it reads are
// the key, the lists' contents are uploaded before each launch
std::vector<long long> graph_key(const Engine* E, const Task2* dt, const SweepPlan& P) {
  std::vector<long long> k = {P.K, P.two, P.n_order, (long long)(uintptr_t)dt, E->max_inner};
  long long tol;
  std::memcpy(&tol, &E->tol_mult, sizeof tol);
  k.push_back(tol);
  for (int i = 0; i < P.K; ++i)
    for (const mpsk::Ent* l : {P.la[i], P.lb[i], P.lo[i]}) k.push_back((long long)(uintptr_t)l);
  for (const SweepGroup& g : P.groups)
    for (long long v : {g.bw, g.inner_few, g.na, g.nb, g.oa, g.ob, g.mNa, g.mNb, (int)g.split_a, (int)g.split_b})
      k.push_back(v);
  return k;
}

hipError_t launch_sweep_graph(Engine* E, Task2* dt, const SweepPlan& P, hipStream_t st) {
  const std::vector<long long> key = graph_key(E, dt, P);
  auto it = E->graphs.find(key);
  if (it == E->graphs.end()) {
    if (E->graphs.size() >= 256) {  // shapes come and go with the workload: start over
      for (auto& kv : E->graphs) (void)hipGraphExecDestroy(kv.second);
      E->graphs.clear();
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    const hipError_t ec = enqueue_sweeps(E, dt, P, st);
    e = hipStreamEndCapture(st, &g);
    if (ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return ec;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    it = E->graphs.emplace(key, x).first;
    ++E->graphs_built;
  }
  ++E->graph_launches;
  return hipGraphLaunch(it->second, st);
}

// Runs `gates` on the states `U` of engine E.  d_dims / dims_total: one device range
// covering every state's bond-dimension table; dims_off[u] = offset of state u's.
int run_sched(Engine* E, const std::vector<mps_state*>& U, const int* d_dims, int dims_total,
              const std::vector<int>& dims_off, const std::vector<GateRef>& gates, std::string* err) {
  if (gates.empty()) return MPS_OK;
  // a previous run that ended in an error may have left QR factorisations or dd work
  // queued: let them drain before any slot, list or workspace is reused
  HIPCHK(err, hipStreamSynchronize(E->stream3));
  HIPCHK(err, hipStreamSynchronize(E->stream4));
  const bool dd = E->prec == MPS_PREC_DD;
  const int nu = (int)U.size();
  std::vector<int> site_base(nu + 1, 0);
  for (int u = 0; u < nu; ++u) site_base[u + 1] = site_base[u] + U[u]->n;
  const int nsites = site_base[nu];
  std::vector<std::vector<int>> queue(nu);
  int n2 = 0, n3 = 0, par = 0;
  size_t max_need = 0;
  int capmax = 1;
  for (int u = 0; u < nu; ++u) {
    par += std::max(2, U[u]->n / 2 + 1);
    for (int b = 0; b <= U[u]->n; ++b) capmax = std::max(capmax, U[u]->capx[b]);
  }
  for (size_t gi = 0; gi < gates.size(); ++gi) {
    const GateRef& g = gates[gi];
    queue[g.unit].push_back((int)gi);
    n2 += g.k == 2;
    n3 += g.k == 3;
    max_need = std::max(max_need, gate_need_cap(dd, U[g.unit], g.first, g.k));
  }
  const int S = std::max(n3 ? 2 : 1, std::min(std::min(E->max_slots, par), std::max(1, n2 + 2 * n3)));
  // standalone engines: every slot takes the same, largest workspace (no
  // fragmentation); batch engines: each update takes what its shape needs
  size_t uniform = 0, arena_bytes;
  if (!E->batch) {
    const int Mcap = 2 * capmax, Ncap = (n3 ? 4 : 2) * capmax;
    uniform = task_ws_bound(dd, Mcap, Ncap, n3 ? 4 * capmax * capmax : 0);
    arena_bytes = uniform * S;
  } else {
    arena_bytes = std::max(max_need, (size_t)std::min(E->ws_limit, (double)max_need * S));
  }
  int rc = ensure_ws(E, align_up(arena_bytes), err);
  if (rc) return rc;
  // small device / pinned areas
  const size_t o_tasks = 0;
  const size_t o_flags = align_up(sizeof(Task2) * S);
  const size_t o_stats = o_flags + align_up(sizeof(int) * 3 * S);
  const size_t o_fro = o_stats + align_up(sizeof(double) * 8 * S);
  const size_t o_dims = o_fro + align_up(sizeof(double) * S);
  const size_t o_u8 = o_dims + align_up(sizeof(int) * dims_total);
  const size_t o_g1 = o_u8 + align_up(sizeof(double2) * 128 * S);
  const size_t o_ents = o_g1 + align_up(sizeof(Task1) * nsites);
  // new2, new3, jacobi (two halves + order, for each of two sweeps), dd, dd-enter,
  // final, final3, mid, znorm, ref, polish, qr z, dd-enter QR tasks, and a ring of
  // kQrRing lists of QR factorisations in flight
  constexpr int kQrRing = 4;
  constexpr int kLists = 18 + kQrRing;
  const size_t list_bytes = align_up(sizeof(mpsk::Ent) * S);
  rc = ensure_small(E, o_ents + kLists * list_bytes, err);
  if (rc) return rc;
  Task2* ht = (Task2*)(E->h_stage + o_tasks);
  Task2* dt = (Task2*)(E->d_small + o_tasks);
  int* d_flags = (int*)(E->d_small + o_flags);
  int* hflags = (int*)(E->h_stage + o_flags);
  double* d_stats = (double*)(E->d_small + o_stats);
  double* hstats = (double*)(E->h_stage + o_stats);
  double* d_fro = (double*)(E->d_small + o_fro);
  int* hdims = (int*)(E->h_stage + o_dims);
  double2* hu8 = (double2*)(E->h_stage + o_u8);
  double2* du8 = (double2*)(E->d_small + o_u8);
  enum { LN2 = 0, LN3, LJ, LD, LENTER, LFIN, LFIN3, LMID, LZN, LR, LPOL, LJ2, LJO, LQZ, LQL, LJ_1, LJ2_1, LJO_1, LQR0 };
  auto hlist = [&](int i) { return E->h_stage + o_ents + i * list_bytes; };
  auto dlist = [&](int i) { return E->d_small + o_ents + i * list_bytes; };

  std::vector<Slot> slot(S);
  std::vector<char> done(gates.size(), 0), busy(nsites, 0), claimed(nsites, 0);
  std::vector<double> gstats(8 * gates.size(), 0.0);
  std::vector<int> gsweeps(gates.size(), 0), gdd(gates.size(), 0);
  std::vector<size_t> head(nu, 0);  // per state: first queue entry not yet admitted
  size_t remaining = gates.size();
  int status = MPS_OK;
  int rot0 = 0;  // first state scanned at admission (rotates for fairness)
  hipError_t e;
  hipStream_t st = E->stream;
  // the dd work's stream; its launches follow everything queued on st so far (fork)
  // and st waits for them before reading flags back (join)
  hipStream_t sd = (dd && E->dd_stream) ? E->stream4 : st;
  bool sd_pending = false;
  auto fork_dd = [&]() -> hipError_t {
    if (sd == st) return hipSuccess;
    hipError_t ee = hipEventRecord(E->ev_dd_fork, st);
    if (ee == hipSuccess) ee = hipStreamWaitEvent(sd, E->ev_dd_fork, 0);
    sd_pending = true;
    return ee;
  };
  auto join_dd = [&]() -> hipError_t {
    if (!sd_pending) return hipSuccess;
    sd_pending = false;
    hipError_t ee = hipEventRecord(E->ev_dd_join, sd);
    if (ee == hipSuccess) ee = hipStreamWaitEvent(st, E->ev_dd_join, 0);
    return ee;
  };
  int dirty_lo = S, dirty_hi = -1;  // task descriptors changed since the last upload
  auto mark = [&](int si) { dirty_lo = std::min(dirty_lo, si); dirty_hi = std::max(dirty_hi, si); };
  auto upload_tasks = [&]() -> hipError_t {
    if (dirty_hi < dirty_lo) return hipSuccess;
    hipError_t ee = hipMemcpyAsync(dt + dirty_lo, ht + dirty_lo, sizeof(Task2) * (dirty_hi - dirty_lo + 1),
                                   hipMemcpyHostToDevice, st);
    dirty_lo = S;
    dirty_hi = -1;
    return ee;
  };

  auto upload_list = [&](int li, const std::vector<mpsk::Ent>& ents) -> mpsk::Ent* {
    mpsk::Ent* hl = (mpsk::Ent*)hlist(li);
    for (size_t i = 0; i < ents.size(); ++i) hl[i] = ents[i];
    hipError_t ee = hipMemcpyAsync(dlist(li), hl, sizeof(mpsk::Ent) * ents.size(), hipMemcpyHostToDevice, st);
    return ee == hipSuccess ? (mpsk::Ent*)dlist(li) : nullptr;
  };
  auto ents_of = [&](const std::vector<int>& sl) {
    std::vector<mpsk::Ent> v;
    v.reserve(sl.size());
    for (int si : sl) v.push_back(mpsk::Ent{si, slot[si].sweep});
    return v;
  };
  // the FP64 sweeps of the iterating slots `jl` (K of them), as stream launches or
  // as a replayed graph
  auto launch_jacobi = [&](const std::vector<int>& jl, int K) -> hipError_t {
    SweepPlan P;
    P.K = K;
    P.two = E->jacobi_streams == 2 && jl.size() >= 2;
    P.n_order = (int)jl.size();
    // groups by step kernel configuration, in order of first appearance
    std::vector<std::vector<int>> ga, gb;
    std::vector<std::pair<int, int>> cfgs;
    for (int si : jl) {
      const std::pair<int, int> c{slot[si].bw, slot[si].inner_few};
      size_t gi = 0;
      while (gi < cfgs.size() && cfgs[gi] != c) ++gi;
      if (gi == cfgs.size()) {
        cfgs.push_back(c);
        ga.emplace_back();
        gb.emplace_back();
      }
      // alternate updates of a group go to the two halves
      ((P.two && ((ga[gi].size() + gb[gi].size()) & 1)) ? gb[gi] : ga[gi]).push_back(si);
    }
    std::vector<int> all_a, all_b;
    for (size_t gi = 0; gi < cfgs.size(); ++gi) {
      SweepGroup g;
      g.bw = cfgs[gi].first;
      g.inner_few = cfgs[gi].second;
      g.na = (int)ga[gi].size();
      g.nb = (int)gb[gi].size();
      g.oa = (int)all_a.size();
      g.ob = (int)all_b.size();
      for (int si : ga[gi]) g.mNa = std::max(g.mNa, slot[si].N);
      for (int si : gb[gi]) g.mNb = std::max(g.mNb, slot[si].N);
      g.split_a = g.bw == 8 && g.na <= E->split_max;
      g.split_b = g.bw == 8 && g.nb <= E->split_max;
      all_a.insert(all_a.end(), ga[gi].begin(), ga[gi].end());
      all_b.insert(all_b.end(), gb[gi].begin(), gb[gi].end());
      P.groups.push_back(g);
    }
    const int lists[2][3] = {{LJ, LJ2, LJO}, {LJ_1, LJ2_1, LJO_1}};
    for (int k = 0; k < K; ++k) {
      auto with_sweep = [&](const std::vector<int>& v) {
        std::vector<mpsk::Ent> out = ents_of(v);
        for (mpsk::Ent& x : out) x.sweep += k;
        return out;
      };
      P.la[k] = upload_list(lists[k][0], with_sweep(all_a));
      P.lb[k] = all_b.empty() ? P.la[k] : upload_list(lists[k][1], with_sweep(all_b));
      P.lo[k] = upload_list(lists[k][2], with_sweep(jl));
      if (!P.la[k] || !P.lb[k] || !P.lo[k]) return hipErrorInvalidValue;
    }
    P.phase = E->d_phase;
    Timed tm(E, 1, K * plan_steps(P));
    if (E->graphs_on && !E->d_phase) return launch_sweep_graph(E, dt, P, st);
    return enqueue_sweeps(E, dt, P, st);
  };
  std::vector<int> free_list;  // free slot indices, lowest last
  for (int si = S - 1; si >= 0; --si) free_list.push_back(si);
  auto take_slot = [&]() {
    const int si = free_list.back();
    free_list.pop_back();
    return si;
  };
  auto release_slot = [&](int si) {
    if (slot[si].ws_len) E->arena.release(slot[si].ws_off, slot[si].ws_len);
    slot[si] = Slot{};
    free_list.push_back(si);
  };
  auto ws_alloc = [&](size_t need, size_t& off) {
    const size_t len = align_up(uniform ? uniform : need);
    off = E->arena.alloc(len);
    return off == SIZE_MAX ? (size_t)0 : len;
  };
  std::vector<int> active;  // slots not free

  bool unsynced = false;  // async copies from the pinned staging may still be pending
  // QR factorisations in flight on stream3, oldest first: completion event, list ring
  // slot, the slots waiting (state 6); polled at the end of each tick, so that a
  // factorisation longer than a sweep does not hold up the other updates' sweeps
  struct QrBatch {
    hipEvent_t ev;
    std::vector<int> slots;
  };
  std::deque<QrBatch> qr_inflight;
  int qr_ring = 0;
  auto qr_poll = [&](bool block) -> hipError_t {
    while (!qr_inflight.empty()) {
      QrBatch& b = qr_inflight.front();
      const hipError_t q = block ? hipEventSynchronize(b.ev) : hipEventQuery(b.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return q;
      for (int si : b.slots)
        if (slot[si].state == 6) slot[si].state = 1;
      E->evpool.push_back(b.ev);
      qr_inflight.pop_front();
      if (block) block = false;  // one finished batch is progress enough
    }
    return hipSuccess;
  };
  while (true) {
    // the staging buffers are rewritten below: wait for copies a previous tick left
    if (unsynced) {
      HIPCHK(err, hipStreamSynchronize(st));
      unsynced = false;
    }
    // ---- 1. admission
    std::vector<int> new2, new3;
    std::vector<Task1> g1;
    long g1_maxel = 0;
    std::fill(claimed.begin(), claimed.end(), 0);
    for (int uu = 0; uu < nu && remaining; ++uu) {
      const int u = (rot0 + uu) % nu;
      const mps_state* h = U[u];
      const int sb0 = site_base[u];
      std::vector<int>& qu = queue[u];
      while (head[u] < qu.size() && done[qu[head[u]]]) ++head[u];
      int blocked = 0;  // sites of this state that no later gate may use this tick
      for (int q = 0; q < h->n; ++q) blocked += busy[sb0 + q];
      const size_t window = (size_t)4 * h->n + 16;
      for (size_t qi = head[u]; qi < qu.size() && qi < head[u] + window && blocked < h->n; ++qi) {
        const int gi = qu[qi];
        if (done[gi]) continue;
        const GateRef& g = gates[gi];
        bool free_ = true;
        for (int q = g.first; q < g.first + g.k; ++q) free_ &= !busy[sb0 + q] && !claimed[sb0 + q];
        if (free_ && g.k == 1) {
          Task1 t{};
          t.B = h->B[g.first];
          t.B_lo = dd ? h->Blo[g.first] : nullptr;
          t.ld = h->capx[g.first + 1];
          t.a = h->dimx[g.first];
          t.b = h->dimx[g.first + 1];
          for (int q = 0; q < 4; ++q) {
            t.U[q] = make_double2(g.U[2 * q], g.U[2 * q + 1]);
            t.U_lo[q] = (dd && g.Ulo) ? make_double2(g.Ulo[2 * q], g.Ulo[2 * q + 1]) : make_double2(0, 0);
          }
          g1.push_back(t);
          g1_maxel = std::max(g1_maxel, (long)t.a * t.b);
          done[gi] = 1;
          --remaining;
          claimed[sb0 + g.first] = 1;  // later gates on this site wait for the next tick
          ++blocked;
          continue;
        }
        const int s0 = g.first;
        bool admitted = false;
        if (free_ && (int)free_list.size() >= (g.k == 3 ? 2 : 1)) {
          size_t off1 = 0, off2 = 0, len1 = 0, len2 = 0;
          if (g.k == 2) {
            len1 = ws_alloc(task_ws_bytes(dd, 2 * h->dimx[s0], 2 * h->dimx[s0 + 2], 0), off1);
          } else {
            const int a = h->dimx[s0], c = h->dimx[s0 + 2], d = h->dimx[s0 + 3];
            len1 = ws_alloc(task_ws_bytes(dd, 2 * a, 4 * d, 4 * a * c), off1);
            if (len1) {
              len2 = ws_alloc(task_ws_bound(dd, 2 * h->capx[s0 + 1], 2 * d, 0), off2);
              if (!len2) {
                E->arena.release(off1, len1);
                len1 = 0;
              }
            }
          }
          if (len1) {
            admitted = true;
            const int si = take_slot();
            Slot& sl = slot[si];
            sl = Slot{};
            sl.state = 1;
            sl.gate = gi;
            sl.ws_off = off1;
            sl.ws_len = len1;
            Task2& t = ht[si];
            setup_split(h, t, s0, h->dimx[s0], h->dimx[s0 + 1], h->dimx[s0 + 2]);
            if (g.k == 2) {
              for (int q = 0; q < 16; ++q) {
                t.U[q] = make_double2(g.U[2 * q], g.U[2 * q + 1]);
                t.U_lo[q] = (dd && g.Ulo) ? make_double2(g.Ulo[2 * q], g.Ulo[2 * q + 1]) : make_double2(0, 0);
              }
              new2.push_back(si);
            } else {
              t.B3 = h->B[s0 + 2];
              t.B3_lo = dd ? h->Blo[s0 + 2] : nullptr;
              t.ld3 = h->capx[s0 + 3];
              t.d = h->dimx[s0 + 3];
              set_cols(t, 4 * t.d);
              double2* u8h = hu8 + 128 * si;
              for (int q = 0; q < 64; ++q) {
                u8h[q] = make_double2(g.U[2 * q], g.U[2 * q + 1]);
                u8h[64 + q] = (dd && g.Ulo) ? make_double2(g.Ulo[2 * q], g.Ulo[2 * q + 1]) : make_double2(0, 0);
              }
              t.U8 = du8 + 128 * si;
              t.U8_lo = du8 + 128 * si + 64;
              sl.kind = 1;
              const int sb = take_slot();
              slot[sb] = Slot{};
              slot[sb].state = 5;
              slot[sb].kind = 2;
              slot[sb].gate = gi;
              slot[sb].ws_off = off2;
              slot[sb].ws_len = len2;
              sl.partner = sb;
              active.push_back(sb);
              new3.push_back(si);
            }
            carve(dd, t, E->ws + off1, d_flags, d_stats, d_fro, si);
            const StepCfg cfg = step_cfg(E, t.N);
            sl.bw = cfg.bw;
            sl.inner_few = cfg.inner_few;
            if (g.k == 2 && cfg.qr) qr_select(dd, t);
            if (t.qr) sl.state = 6;  // waits one tick for its QR factorisation
            mark(si);
            sl.M = t.M;
            sl.N = t.N;
            sl.Nt = t.Nt;
            sl.JM = t.JM;
            active.push_back(si);
            for (int q = g.first; q < g.first + g.k; ++q) busy[sb0 + q] = 1;
            done[gi] = 1;
            --remaining;
          }
        }
        if (!admitted)
          for (int q = g.first; q < g.first + g.k; ++q) {
            blocked += !claimed[sb0 + q] && !busy[sb0 + q];
            claimed[sb0 + q] = 1;
          }
        else
          blocked += g.k;
      }
    }
    rot0 = nu ? (rot0 + 1) % nu : 0;
    if (!g1.empty()) {
      Task1* h1 = (Task1*)(E->h_stage + o_g1);
      std::memcpy(h1, g1.data(), sizeof(Task1) * g1.size());
      HIPCHK(err, hipMemcpyAsync(E->d_small + o_g1, h1, sizeof(Task1) * g1.size(), hipMemcpyHostToDevice, st));
      unsynced = true;
      Timed tm(E, 4);
      e = dd ? mpsk::launch_gate1_dd((Task1*)(E->d_small + o_g1), (int)g1.size(), g1_maxel, st)
             : mpsk::launch_gate1((Task1*)(E->d_small + o_g1), (int)g1.size(), g1_maxel, st);
      if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("gate1: ") + hipGetErrorString(e));
    }
    if (!new2.empty() || !new3.empty()) {
      HIPCHK(err, upload_tasks());
      if (!new3.empty())
        for (int si : new3)
          HIPCHK(err, hipMemcpyAsync(du8 + 128 * si, hu8 + 128 * si, sizeof(double2) * 128, hipMemcpyHostToDevice, st));
      unsynced = true;
      for (int which = 0; which < 2; ++which) {
        Timed tm(E, 0);
        const std::vector<int>& nl = which ? new3 : new2;
        if (nl.empty()) continue;
        mpsk::Ent* el = upload_list(which ? LN3 : LN2, ents_of(nl));
        if (!el) return fail(err, MPS_EDEVICE, "list upload failed");
        int mM = 0, mN = 0, mNt = 0, mA = 0, mC = 0, mD = 0;
        for (int si : nl) {
          mM = std::max(mM, slot[si].M);
          mN = std::max(mN, slot[si].N);
          mNt = std::max(mNt, slot[si].Nt);
          mA = std::max(mA, ht[si].a);
          mC = std::max(mC, ht[si].c);
          mD = std::max(mD, ht[si].d);
        }
        e = mpsk::launch_prep2(dt, el, (int)nl.size(), mN, st);
        if (e == hipSuccess) {
          if (which)
            e = mpsk::launch_theta3(dt, el, (int)nl.size(), mA, mC, mD, dd, st);
          else
            e = dd ? mpsk::launch_theta2_dd(dt, el, (int)nl.size(), mM, mNt, st)
                   : mpsk::launch_theta2(dt, el, (int)nl.size(), mM, mNt, st);
        }
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("theta: ") + hipGetErrorString(e));
        std::vector<int> qrs;
        for (int si : nl)
          if (ht[si].qr) qrs.push_back(si);
        if (!qrs.empty()) {  // on stream3 after the theta kernels, with a list of its own
          if ((int)qr_inflight.size() >= kQrRing) HIPCHK(err, qr_poll(true));  // frees the oldest ring slot
          mpsk::Ent* eq = upload_list(LQR0 + qr_ring, ents_of(qrs));
          if (!eq) return fail(err, MPS_EDEVICE, "list upload failed");
          qr_ring = (qr_ring + 1) % kQrRing;
          HIPCHK(err, hipEventRecord(E->ev_qr, st));
          HIPCHK(err, hipStreamWaitEvent(E->stream3, E->ev_qr, 0));
          e = mpsk::launch_qr_factor(dt, eq, (int)qrs.size(), mM, mN, E->stream3);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("qr: ") + hipGetErrorString(e));
          hipEvent_t done = ev_get(E);
          if (!done) return fail(err, MPS_EDEVICE, "event creation failed");
          HIPCHK(err, hipEventRecord(done, E->stream3));
          qr_inflight.push_back(QrBatch{done, qrs});
        }
      }
    }
    // ---- 2. one sweep for every iterating slot (QR-pending slots wait)
    std::vector<int> jl, rl, dl;
    for (int si : active) {
      if (slot[si].state == 1) jl.push_back(si);
      if (slot[si].state == 2) rl.push_back(si);
      if (slot[si].state == 4) dl.push_back(si);
    }
    if (jl.empty() && rl.empty() && dl.empty() && qr_inflight.empty()) {
      if (active.empty()) {
        if (!remaining) break;
        continue;  // only single-site gates were admitted; admit the rest
      }
    }
    // dd refinement passes and polish sweeps first, on the dd stream, so that they
    // overlap the FP64 sweeps launched below
    if (!rl.empty() || !dl.empty()) {
      mpsk::Ent* elr = rl.empty() ? nullptr : upload_list(LR, ents_of(rl));
      mpsk::Ent* eld = dl.empty() ? nullptr : upload_list(LD, ents_of(dl));
      if ((!rl.empty() && !elr) || (!dl.empty() && !eld)) return fail(err, MPS_EDEVICE, "list upload failed");
      HIPCHK(err, fork_dd());
      if (!rl.empty()) {
        int mM = 0, mN = 0;
        for (int si : rl) { mM = std::max(mM, slot[si].JM); mN = std::max(mN, slot[si].N); }
        Timed tm(E, 6, 1, sd);
        E->slot_sweeps_dd += (long)rl.size();
        e = mpsk::launch_ddref_pass(dt, elr, (int)rl.size(), mM, mN, E->tol_mult, sd);
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("dd refinement: ") + hipGetErrorString(e));
      }
      if (!dl.empty()) {
        int mN = 0;
        for (int si : dl) mN = std::max(mN, slot[si].N);
        const int nb = (mN + 7) / 8;
        const int nsteps = nb + (nb & 1) - 1;
        Timed tm(E, 6, nsteps, sd);
        E->slot_sweeps_dd += (long)dl.size();
        for (int stp = 0; stp < nsteps; ++stp) {
          e = mpsk::launch_jacobi_step_dd(dt, eld, (int)dl.size(), mN, stp, E->tol_mult, E->max_inner, sd);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("dd jacobi: ") + hipGetErrorString(e));
        }
      }
    }
    int K = 1;  // sweeps this tick
    if (!jl.empty()) {
      K = std::max(1, std::min(2, E->tick_sweeps));
      for (int si : jl) K = std::min(K, E->max_sweeps - slot[si].sweep);
      K = std::max(K, 1);
      HIPCHK(err, launch_jacobi(jl, K));
    }
    // finished QR factorisations: their slots start iterating at the next tick; when
    // this tick has no sweep work at all, wait for the oldest
    HIPCHK(err, qr_poll(jl.empty() && rl.empty() && dl.empty()));
    // ---- 3. convergence
    HIPCHK(err, join_dd());
    if (!jl.empty() || !rl.empty() || !dl.empty()) {
      HIPCHK(err, hipMemcpyAsync(hflags, d_flags, sizeof(int) * 3 * S, hipMemcpyDeviceToHost, st));
      HIPCHK(err, hipStreamSynchronize(st));
      unsynced = false;
      if (E->d_phase && !jl.empty()) {
        long long pc[5];
        HIPCHK(err, hipMemcpy(pc, E->d_phase, sizeof(pc), hipMemcpyDeviceToHost));
        // wall_clock64 runs at 100 MHz on gfx950
        std::fprintf(stderr, "[mps] step phases (us, %zu updates, N %d): gram %.1f inner %.1f update %.1f rot %lld\n",
                     jl.size(), slot[jl[0]].N, (pc[1] - pc[0]) * 0.01, (pc[2] - pc[1]) * 0.01, (pc[3] - pc[2]) * 0.01,
                     pc[4]);
      }
    }
    std::vector<int> enter;
    for (int si : jl) {
      Slot& sl = slot[si];
      // the tick's K sweeps: the first without a rotation ends the iteration (the
      // sweeps after it left the update untouched)
      bool rot = true;
      for (int k = 0; k < K && rot; ++k) {
        rot = hflags[3 * si + sl.sweep % 3] != 0;
        ++sl.sweep;
        ++E->slot_sweeps;
      }
      if (!rot || sl.sweep >= E->max_sweeps) {
        sl.fp64_sweeps = sl.sweep;
        sl.fp64_conv = !rot;
        if (dd) {
          enter.push_back(si);
          sl.state = E->dd_refine ? 2 : 4;
          sl.sweep = 0;
        } else {
          sl.conv = sl.fp64_conv;
          sl.state = 3;
        }
      }
    }
    std::vector<int> to_polish;
    for (int si : rl) {
      Slot& sl = slot[si];
      const int code = hflags[3 * si + sl.sweep % 3];
      ++sl.sweep;
      if (code == 0) {
        sl.dd_sweeps = sl.sweep;
        sl.conv = true;
        sl.state = 3;
      } else if ((code & 2) || sl.sweep >= E->max_ref_passes) {
        sl.dd_sweeps = sl.sweep;
        sl.state = 4;
        sl.sweep = 0;
        to_polish.push_back(si);
      }
    }
    for (int si : dl) {
      Slot& sl = slot[si];
      const bool rot = hflags[3 * si + sl.sweep % 3] != 0;
      ++sl.sweep;
      if (!rot || sl.sweep >= E->max_sweeps_dd) {
        sl.dd_sweeps += sl.sweep;
        sl.conv = !rot;
        sl.state = 3;
      }
    }
    if (!to_polish.empty()) {
      unsynced = true;
      mpsk::Ent* el = upload_list(LPOL, ents_of(to_polish));
      if (!el) return fail(err, MPS_EDEVICE, "list upload failed");
      HIPCHK(err, fork_dd());
      e = mpsk::launch_flags_clear(dt, el, (int)to_polish.size(), sd);
      if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("flags: ") + hipGetErrorString(e));
    }
    if (!enter.empty()) {
      unsynced = true;
      mpsk::Ent* el = upload_list(LENTER, ents_of(enter));
      if (!el) return fail(err, MPS_EDEVICE, "list upload failed");
      // QR-preconditioned tasks: V <- Q V_x, then the refinement of the transposed
      // problem (square thetas: the shapes stay the same).  The descriptors are
      // converted first; the Q application reads none of the converted fields, so it
      // and the promotion both follow the upload on the dd stream.
      std::vector<int> qrl;
      int qN = 0;
      for (int si : enter)
        if (ht[si].qr) {
          qrl.push_back(si);
          qN = std::max(qN, ht[si].N);
        }
      mpsk::Ent* eql = nullptr;
      if (!qrl.empty()) {
        eql = upload_list(LQL, ents_of(qrl));
        if (!eql) return fail(err, MPS_EDEVICE, "list upload failed");
        for (int si : qrl) {
          qr_to_transposed(ht[si]);
          slot[si].JM = ht[si].JM;
          slot[si].N = ht[si].N;
          mark(si);
        }
        HIPCHK(err, upload_tasks());
      }
      int mM = 0, mN = 0;
      for (int si : enter) { mM = std::max(mM, slot[si].JM); mN = std::max(mN, slot[si].N); }
      HIPCHK(err, fork_dd());
      if (eql) {
        Timed tq(E, 6, 1, sd);
        e = mpsk::launch_qr_left(dt, eql, (int)qrl.size(), qN, sd);
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("qr left: ") + hipGetErrorString(e));
      }
      Timed tm(E, 6, 1, sd);
      e = mpsk::launch_dd_enter(dt, el, (int)enter.size(), mM, mN, sd);
      if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("dd enter: ") + hipGetErrorString(e));
    }
    // ---- 4. finalise converged slots
    std::vector<int> fl, fl2, fl3;
    for (int si : active)
      if (slot[si].state == 3) {
        fl.push_back(si);
        (slot[si].kind == 1 ? fl3 : fl2).push_back(si);
      }
    if (!fl.empty()) {
      mpsk::Ent* el = upload_list(LFIN, ents_of(fl));
      if (!el) return fail(err, MPS_EDEVICE, "list upload failed");
      {
        Timed tm(E, 2);
        e = dd ? mpsk::launch_truncate_dd(dt, el, (int)fl.size(), E->rank_floor_dd, st)
               : mpsk::launch_truncate(dt, el, (int)fl.size(), E->rank_floor, st);
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("truncate: ") + hipGetErrorString(e));
      }
      {
        std::vector<int> zl;
        int zJM = 0, zK = 1;
        for (int si : fl)
          if (ht[si].tr) {
            zl.push_back(si);
            zJM = std::max(zJM, ht[si].JM);
            zK = std::max(zK, std::min(ht[si].chi, ht[si].N));
          }
        if (!zl.empty()) {
          mpsk::Ent* ez = upload_list(LZN, ents_of(zl));
          if (!ez) return fail(err, MPS_EDEVICE, "list upload failed");
          Timed tz(E, 3);
          e = dd ? mpsk::launch_znorm_dd(dt, ez, (int)zl.size(), zJM, zK, st)
                 : mpsk::launch_znorm(dt, ez, (int)zl.size(), zJM, zK, st);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("znorm: ") + hipGetErrorString(e));
        }
        std::vector<int> ql;  // FP64 tasks preconditioned by QR: Z from W's columns
        int qN = 0, qK = 1;
        for (int si : fl)
          if (ht[si].qr) {
            ql.push_back(si);
            qN = std::max(qN, ht[si].N);
            qK = std::max(qK, std::min(ht[si].chi, ht[si].N));
          }
        if (!ql.empty()) {
          mpsk::Ent* eq = upload_list(LQZ, ents_of(ql));
          if (!eq) return fail(err, MPS_EDEVICE, "list upload failed");
          Timed tz(E, 3);
          e = mpsk::launch_qr_z(dt, eq, (int)ql.size(), qN, qK, st);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("qr z: ") + hipGetErrorString(e));
        }
      }
      {
        Timed tm(E, 3);
        for (int which = 0; which < 2; ++which) {
          const std::vector<int>& ll = which ? fl3 : fl2;
          if (ll.empty()) continue;
          mpsk::Ent* e2 = which ? upload_list(LFIN3, ents_of(ll)) : upload_list(LMID, ents_of(ll));
          if (!e2) return fail(err, MPS_EDEVICE, "list upload failed");
          int lM = 0, lN = 0, maxK = 1;
          for (int si : ll) {
            lM = std::max(lM, slot[si].M);
            lN = std::max(lN, slot[si].Nt);
            maxK = std::max(maxK, std::min(ht[si].chi, std::min(slot[si].M, slot[si].N)));
          }
          e = dd ? mpsk::launch_split_dd(dt, e2, (int)ll.size(), lM, lN, maxK, st, which == 0)
                 : mpsk::launch_split(dt, e2, (int)ll.size(), lM, lN, maxK, st, which == 0);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("split: ") + hipGetErrorString(e));
        }
      }
      HIPCHK(err, hipMemcpyAsync(hstats, d_stats, sizeof(double) * 8 * S, hipMemcpyDeviceToHost, st));
      HIPCHK(err, hipMemcpyAsync(hdims, d_dims, sizeof(int) * dims_total, hipMemcpyDeviceToHost, st));
      HIPCHK(err, hipStreamSynchronize(st));
      unsynced = false;
      for (int u = 0; u < nu; ++u) std::memcpy(U[u]->dimx.data(), hdims + dims_off[u], sizeof(int) * (U[u]->n + 1));
      // first splits of three-site gates: the second split takes over in the reserved slot
      std::vector<mpsk::Ent> mids;
      std::vector<int> newB;
      int mN1 = 0, mK1 = 0, mNB = 0;
      for (int si : fl3) {
        Slot& sa = slot[si];
        const GateRef& g = gates[sa.gate];
        const mps_state* h = U[g.unit];
        const int s0 = g.first, sb = sa.partner;
        Task2& tb = ht[sb];
        setup_split(h, tb, s0 + 1, h->dimx[s0 + 1], 0, h->dimx[s0 + 3]);
        carve(dd, tb, E->ws + slot[sb].ws_off, d_flags, d_stats, d_fro, sb);
        mark(sb);
        Slot& sbl = slot[sb];
        sbl.state = 1;
        sbl.sweep = 0;
        sbl.M = tb.M;
        sbl.N = tb.N;
        const StepCfg cfg = step_cfg(E, tb.N);
        sbl.bw = cfg.bw;
        sbl.inner_few = cfg.inner_few;
        sbl.Nt = tb.Nt;
        sbl.JM = tb.JM;
        gsweeps[sa.gate] = sa.fp64_sweeps;
        gdd[sa.gate] = sa.dd_sweeps;
        if (!sa.conv) {
          status = MPS_ENOCONV;
          ++E->noconv_updates;
        }
        mids.push_back(mpsk::Ent{si, sb});
        newB.push_back(sb);
        mN1 = std::max(mN1, sa.Nt);
        mK1 = std::max(mK1, std::min(h->chi, sa.M));
        mNB = std::max(mNB, tb.N);
      }
      if (!mids.empty()) {
        HIPCHK(err, upload_tasks());
        unsynced = true;
        mpsk::Ent* eb = upload_list(LN2, ents_of(newB));
        mpsk::Ent* em = upload_list(LN3, mids);
        if (!eb || !em) return fail(err, MPS_EDEVICE, "list upload failed");
        {
          Timed tm(E, 0);
          e = mpsk::launch_prep2(dt, eb, (int)newB.size(), mNB, st);
          if (e == hipSuccess) e = mpsk::launch_mid3(dt, em, (int)mids.size(), mN1, mK1, dd, st);
          if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("mid: ") + hipGetErrorString(e));
        }
      }
      // a released slot's workspace is reused only by launches queued after the
      // kernels that still read it (one stream)
      for (int si : fl3) release_slot(si);
      for (int si : fl2) {
        Slot& sl = slot[si];
        const GateRef& g = gates[sl.gate];
        std::memcpy(&gstats[8 * sl.gate], hstats + 8 * si, sizeof(double) * 8);
        gsweeps[sl.gate] = std::max(gsweeps[sl.gate], sl.fp64_sweeps);
        gdd[sl.gate] = std::max(gdd[sl.gate], sl.dd_sweeps);
        if (!sl.conv) {
          status = MPS_ENOCONV;
          ++E->noconv_updates;
        }
        if (E->debug_sweeps)
          std::fprintf(stderr, "[mps] update at state %d site %d (M %d, N %d, kind %d): %d FP64 sweeps, %d dd sweeps\n",
                       g.unit, g.first, sl.M, sl.N, sl.kind, sl.fp64_sweeps, sl.dd_sweeps);
        for (int q = g.first; q < g.first + g.k; ++q) busy[site_base[g.unit] + q] = 0;
        release_slot(si);
      }
      active.erase(std::remove_if(active.begin(), active.end(), [&](int si) { return slot[si].state == 0; }),
                   active.end());
    }
  }
  HIPCHK(err, join_dd());
  HIPCHK(err, hipStreamSynchronize(st));
  for (QrBatch& b : qr_inflight) {  // (none is left once every slot has finished)
    HIPCHK(err, hipEventSynchronize(b.ev));
    E->evpool.push_back(b.ev);
  }
  qr_inflight.clear();
  harvest_timing(E);
  // per state: diagnostics of its last multi-site gate in queue order
  for (int u = 0; u < nu; ++u) {
    mps_state* h = U[u];
    for (size_t qi = queue[u].size(); qi-- > 0;) {
      const int gi = queue[u][qi];
      if (gates[gi].k == 1) continue;
      const double* sv = &gstats[8 * gi];
      h->last = mps_update_stats{};
      h->last.W = sv[0];
      h->last.w = sv[1];
      h->last.gap = sv[2];
      h->last.epsdist = sv[3];
      h->last.k = (int)sv[4];
      h->last.rank = (int)sv[5];
      for (int gj : queue[u]) {
        h->last.sweeps = std::max(h->last.sweeps, gsweeps[gj]);
        h->last.dd_sweeps = std::max(h->last.dd_sweeps, gdd[gj]);
      }
      h->last.splits = gates[gi].k - 1;
      break;
    }
  }
  if (status) return fail(err, status, "Jacobi sweep limit reached");
  return MPS_OK;
}

int run_state(mps_state* h, const std::vector<GateRef>& gates) {
  return run_sched(h->E, {h}, h->d_dimx, h->n + 1, {0}, gates, &h->err);
}

int set_option(Engine* E, int prec, int key, double value, std::string* err) {
  switch (key) {
    case MPS_OPT_MAX_SWEEPS:
      if (!(value >= 1 && value <= 1000)) return fail(err, MPS_EINVAL, "max_sweeps out of range");
      E->max_sweeps = (int)value;
      E->max_sweeps_dd = (int)value;
      return MPS_OK;
    case MPS_OPT_JACOBI_TOL:
      if (!(value > 0 && value <= 1e6)) return fail(err, MPS_EINVAL, "jacobi tol out of range");
      E->tol_mult = value;
      return MPS_OK;
    case MPS_OPT_KERNEL_TIMING:
      E->timing = value != 0;
      return MPS_OK;
    case MPS_OPT_BLOCK_WIDTH:
      if (!(value == 4 || value == 8 || value == 16)) return fail(err, MPS_EINVAL, "block width must be 4, 8 or 16");
      E->block_width = (int)value;
      E->tuned = false;
      return MPS_OK;
    case MPS_OPT_MAX_INNER:
      if (!(value >= 1 && value <= 64)) return fail(err, MPS_EINVAL, "inner sweep limit out of range");
      E->max_inner = (int)value;
      return MPS_OK;
    case MPS_OPT_MAX_INNER_FEW:
      if (!(value >= 1 && value <= 64)) return fail(err, MPS_EINVAL, "inner sweep limit out of range");
      E->max_inner_few = (int)value;
      E->tuned = false;
      return MPS_OK;
    case MPS_OPT_RANK_FLOOR:
      if (!(value >= 0 && value < 1)) return fail(err, MPS_EINVAL, "rank floor out of range");
      if (prec == MPS_PREC_DD) E->rank_floor_dd = value; else E->rank_floor = value;
      return MPS_OK;
    case MPS_OPT_MAX_SLOTS:
      if (!(value >= 1 && value <= 65536)) return fail(err, MPS_EINVAL, "slot limit out of range");
      E->max_slots = (int)value;
      return MPS_OK;
    case MPS_OPT_DD_STREAM:
      if (!(value == 0 || value == 1)) return fail(err, MPS_EINVAL, "dd stream switch must be 0 or 1");
      E->dd_stream = value != 0;
      return MPS_OK;
    case MPS_OPT_STEP_SPLIT:
      if (!(value >= 0 && value <= 1 << 20 && value == (double)(int)value))
        return fail(err, MPS_EINVAL, "step split limit must be a non-negative integer");
      E->split_max = (int)value;
      return MPS_OK;
    case MPS_OPT_QR:
      if (!(value == 0 || value == 1)) return fail(err, MPS_EINVAL, "QR switch must be 0 or 1");
      E->qr = value != 0;
      E->tuned = false;
      return MPS_OK;
    case MPS_OPT_FUSE:
      if (!(value == 0 || value == 1)) return fail(err, MPS_EINVAL, "fusion switch must be 0 or 1");
      E->fuse = value != 0;
      return MPS_OK;
    case MPS_OPT_JACOBI_STREAMS:
      if (!(value == 1 || value == 2)) return fail(err, MPS_EINVAL, "Jacobi stream count must be 1 or 2");
      E->jacobi_streams = (int)value;
      return MPS_OK;
    case MPS_OPT_DD_REFINE:
      if (!(value == 0 || value == 1)) return fail(err, MPS_EINVAL, "dd refinement switch must be 0 or 1");
      E->dd_refine = value != 0;
      return MPS_OK;
    case MPS_OPT_TICK_SWEEPS:
      if (!(value == 1 || value == 2)) return fail(err, MPS_EINVAL, "sweeps per tick must be 1 or 2");
      E->tick_sweeps = (int)value;
      return MPS_OK;
    case MPS_OPT_GRAPH:
      if (!(value == 0 || value == 1)) return fail(err, MPS_EINVAL, "graph switch must be 0 or 1");
      E->graphs_on = value != 0;
      return MPS_OK;
    case MPS_OPT_WORKSPACE_MB:
      if (!(value >= 1 && value <= 1 << 22)) return fail(err, MPS_EINVAL, "workspace limit out of range");
      E->ws_limit = value * (1 << 20);
      return MPS_OK;
    default:
      return fail(err, MPS_EINVAL, "unknown option");
  }
}

}  // namespace

// ====================================================================== C ABI
// ------------------------------------------------------------------ gate fusion
// Scanning a gate list in order: a single-site gate whose site lies inside the
// latest earlier gate touching it is multiplied into that gate (it acts after it:
// U' = G U, G embedded in U's window); latest earlier single-site gates on sites of
// a new gate are multiplied into it (U' = U F) and leave the list.  The gates in
// between act on other sites and commute with the moved one, and a unitary on one
// site of a window leaves the Schmidt values of every cut of the window unchanged,
// so truncation picks the same subspace: the state is the same up to rounding.
// (Multi-site gates are never merged: truncating once after their product is not
// truncating after each.)  Each fusion saves a single-site launch.  The products
// are formed in double-double (and rounded to binary64 for FP64 handles).
namespace {

struct FGate {
  int first, k;
  std::vector<dd::ddr> re, im;  // 4^k entries, row-major
  long pos = 0;                 // list position of the gate that holds this slot
};

FGate fgate_from(int first, int k, const double* hi, const double* lo, long pos) {
  FGate g{first, k, {}, {}, pos};
  const int n = 1 << (2 * k);
  g.re.resize(n);
  g.im.resize(n);
  for (int e = 0; e < n; ++e) {
    g.re[e] = dd::ddr{hi[2 * e], lo ? lo[2 * e] : 0.0};
    g.im[e] = dd::ddr{hi[2 * e + 1], lo ? lo[2 * e + 1] : 0.0};
  }
  return g;
}

// g (k_g sites from g.first) as a 2^K x 2^K matrix on the window of K sites from w0
FGate fgate_embed(const FGate& g, int w0, int K) {
  FGate e{w0, K, {}, {}, g.pos};
  const int D = 1 << K, off = g.first - w0, kg = g.k;
  e.re.assign((size_t)D * D, dd::ddr{0.0, 0.0});
  e.im.assign((size_t)D * D, dd::ddr{0.0, 0.0});
  const int sh = K - off - kg, mask = ((1 << kg) - 1) << sh;
  for (int r = 0; r < D; ++r)
    for (int c = 0; c < D; ++c) {
      if ((r & ~mask) != (c & ~mask)) continue;
      const int gr = (r & mask) >> sh, gc = (c & mask) >> sh;
      e.re[(size_t)r * D + c] = g.re[(size_t)gr * (1 << kg) + gc];
      e.im[(size_t)r * D + c] = g.im[(size_t)gr * (1 << kg) + gc];
    }
  return e;
}

// a * b (same window), complex double-double
FGate fgate_mul(const FGate& a, const FGate& b) {
  FGate c{a.first, a.k, {}, {}, a.pos};
  const int D = 1 << a.k;
  c.re.resize((size_t)D * D);
  c.im.resize((size_t)D * D);
  for (int r = 0; r < D; ++r)
    for (int j = 0; j < D; ++j) {
      dd::ddr sr{0.0, 0.0}, si{0.0, 0.0};
      for (int t = 0; t < D; ++t) {
        const dd::ddr ar = a.re[(size_t)r * D + t], ai = a.im[(size_t)r * D + t];
        const dd::ddr br = b.re[(size_t)t * D + j], bi = b.im[(size_t)t * D + j];
        sr = dd::add(sr, dd::add(dd::mul(ar, br), dd::neg(dd::mul(ai, bi))));
        si = dd::add(si, dd::add(dd::mul(ar, bi), dd::mul(ai, br)));
      }
      c.re[(size_t)r * D + j] = sr;
      c.im[(size_t)r * D + j] = si;
    }
  return c;
}

bool overlaps(const FGate& a, const FGate& b) { return a.first < b.first + b.k && b.first < a.first + a.k; }
bool contains(const FGate& outer, const FGate& inner) {
  return outer.first <= inner.first && inner.first + inner.k <= outer.first + outer.k;
}

std::vector<FGate> fuse_gates(std::vector<FGate> in) {
  std::vector<FGate> out;
  for (FGate& g : in) {
    bool absorbed = false;
    while (true) {
      int f = (int)out.size() - 1;
      while (f >= 0 && !overlaps(out[f], g)) --f;
      if (f < 0) break;
      if (g.k == 1 && contains(out[f], g)) {  // g acts after out[f]
        const long keep = out[f].pos;
        out[f] = fgate_mul(fgate_embed(g, out[f].first, out[f].k), out[f]);
        out[f].pos = keep;
        absorbed = true;
        break;
      }
      if (out[f].k == 1 && contains(g, out[f])) {  // out[f] acts before g: fold it in, look again
        const long keep = g.pos;
        g = fgate_mul(g, fgate_embed(out[f], g.first, g.k));
        g.pos = keep;
        out.erase(out.begin() + f);
        continue;
      }
      break;
    }
    if (!absorbed) out.push_back(std::move(g));
  }
  return out;
}

// A gate list (of one or several states), fused state by state and returned in the
// list's order (a fused gate takes the position of the gate whose slot it holds);
// the fused matrices live in hi / lo, which must outlive the returned list.
std::vector<GateRef> fuse_list(const std::vector<GateRef>& gates, bool dd, std::vector<double>& hi,
                               std::vector<double>& lo) {
  if (gates.size() < 2) return gates;
  std::map<int, std::vector<FGate>> per;
  for (size_t i = 0; i < gates.size(); ++i)
    per[gates[i].unit].push_back(fgate_from(gates[i].first, gates[i].k, gates[i].U, gates[i].Ulo, (long)i));
  std::vector<FGate> fg;
  for (auto& kv : per)
    for (FGate& g : fuse_gates(std::move(kv.second))) fg.push_back(std::move(g));
  if (fg.size() == gates.size()) return gates;
  std::sort(fg.begin(), fg.end(), [](const FGate& x, const FGate& y) { return x.pos < y.pos; });
  size_t total = 0;
  for (const FGate& g : fg) total += (size_t)2 << (2 * g.k);
  hi.assign(total, 0.0);
  lo.assign(dd ? total : 0, 0.0);
  std::vector<GateRef> fused;
  fused.reserve(fg.size());
  size_t o = 0;
  for (const FGate& g : fg) {
    const int ne = 1 << (2 * g.k);
    for (int e = 0; e < ne; ++e) {
      hi[o + 2 * e] = g.re[e].hi;
      hi[o + 2 * e + 1] = g.im[e].hi;
      if (dd) {
        lo[o + 2 * e] = g.re[e].lo;
        lo[o + 2 * e + 1] = g.im[e].lo;
      }
    }
    fused.push_back(GateRef{gates[g.pos].unit, g.first, g.k, hi.data() + o, dd ? lo.data() + o : nullptr});
    o += (size_t)2 * ne;
  }
  return fused;
}

}  // namespace

// helpers of mps_apply_gate2 (non-adjacent gates)
namespace {

// entry (r, c) of a 4 x 4 complex row-major matrix, as doubles
inline double& at4(double* u, int r, int c, int part) { return u[(r * 4 + c) * 2 + part]; }

void swap_gate(double* u) {  // |xy> -> |yx>
  std::memset(u, 0, sizeof(double) * 32);
  at4(u, 0, 0, 0) = at4(u, 1, 2, 0) = at4(u, 2, 1, 0) = at4(u, 3, 3, 0) = 1.0;
}

// U with its two qubits exchanged: U'[(y x), (y' x')] = U[(x y), (x' y')]
void reversed_gate(const double* u, double* out) {
  auto sw = [](int i) { return ((i & 1) << 1) | (i >> 1); };
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c)
      for (int part = 0; part < 2; ++part) out[(sw(r) * 4 + sw(c)) * 2 + part] = u[(r * 4 + c) * 2 + part];
}

// U acting on window positions p0 (its first qubit) and p1 of three sites (position 0
// = the window's first site = the most significant bit), identity on the third.
void outer_gate8(const double* u, int p0, int p1, double* out) {
  std::memset(out, 0, sizeof(double) * 128);
  const int pm = 3 - p0 - p1;
  auto bit = [](int x, int p) { return (x >> (2 - p)) & 1; };
  for (int r = 0; r < 8; ++r)
    for (int c = 0; c < 8; ++c) {
      if (bit(r, pm) != bit(c, pm)) continue;
      const int ur = bit(r, p0) * 2 + bit(r, p1), uc = bit(c, p0) * 2 + bit(c, p1);
      out[(r * 8 + c) * 2] = u[(ur * 4 + uc) * 2];
      out[(r * 8 + c) * 2 + 1] = u[(ur * 4 + uc) * 2 + 1];
    }
}

}  // namespace

// ---------------------------------------------------------------- no-allocation amplitudes
// The amplitude kernels' scratch (bitstrings, site-pointer and row-length tables,
// results) in a fixed device array instead of the engine's staging areas, which
// grow by hipMalloc / hipHostMalloc.  Each device holds its own copy at its own
// address, looked up once per device with that device current.
constexpr size_t kNoAllocScratch = size_t(4) << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// the address of `scratch` on device `dev` (looked up on first use); nullptr on error
void* scratch_on(int dev, hipError_t* e) {
  *e = hipSuccess;
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    *e = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if ((*e = hipGetDevice(&cur)) != hipSuccess) return nullptr;
    if (cur != dev && (*e = hipSetDevice(dev)) != hipSuccess) return nullptr;
    void* p = nullptr;
    *e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (*e == hipSuccess) *e = r;
    }
    if (*e != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// scratch layout of one call: bits | site pointers (hi, then lo) | row lengths | results
struct NoAllocLayout {
  size_t ptr, ld, out, end;
};
NoAllocLayout noalloc_layout(long count, int n, bool dd) {
  NoAllocLayout L;
  L.ptr = align_up((size_t)count * n);
  L.ld = L.ptr + align_up(sizeof(void*) * 2 * n);
  L.out = L.ld + align_up(sizeof(int) * n);
  L.end = L.out + align_up((size_t)count * sizeof(double2) * (dd ? 2 : 1));
  return L;
}

// an error of the no-allocation path: the message is written into the handle's
// reserved string (no temporary strings), cut to its capacity
int fail_na(mps_state* h, int code, const char* what, const char* detail = nullptr) {
  std::string& m = h->err;
  m.clear();
  const size_t cap = m.capacity();
  m.append(what, std::min(std::strlen(what), cap));
  if (detail && m.size() + 2 < cap) {
    m.append(": ");
    m.append(detail, std::min(std::strlen(detail), cap - m.size()));
  }
  return code;
}

#define NACHK(h, call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return fail_na(h, MPS_EDEVICE, #call, hipGetErrorString(e_));             \
  } while (0)

}  // namespace

extern "C" {

const char* mps_version(void) { return "mps-mi355x 0.2 (gfx950)"; }

const char* mps_tuning_key(void) {
  static thread_local std::string key;
  int dev = 0;
  key = hipGetDevice(&dev) == hipSuccess ? tuning_key(dev) : std::string();
  return key.c_str();
}

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
  state_shape(h, n, chi_max, eps, prec);
  h->E = engine_new(prec, hip_stream, &g_create_error);
  if (!h->E) {
    delete h;
    return nullptr;
  }
  h->own_engine = true;
  const size_t bytes = state_bytes(h, true);
  hipError_t e = hipMalloc((void**)&h->mem, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(h->mem, 0, bytes, h->E->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("mps_create: ") + hipGetErrorString(e);
    mps_destroy(h);
    return nullptr;
  }
  state_carve(h, h->mem, true);
  if (set_product_states(h->E, {h}, h->d_dimx, n + 1, &g_create_error)) {
    mps_destroy(h);
    return nullptr;
  }
  return h;
}

mps_handle mps_create(int n, int chi_max, double eps) {
  return mps_create_ex(n, chi_max, eps, MPS_PREC_FP64, nullptr);
}

int mps_destroy(mps_handle h) {
  if (!h) return MPS_EINVAL;
  if (h->batch) return fail(h, MPS_ESTATE, "a batch member is destroyed with its batch");
  engine_sync(h->E);
  if (h->mem) (void)hipFree(h->mem);
  if (h->own_engine) engine_free(h->E);
  delete h;
  return MPS_OK;
}

int mps_apply_gates(mps_handle h, int count, const int* first, const int* k, const double* U, const double* U_lo) {
  if (!h) return MPS_EINVAL;
  if (count < 0 || (count > 0 && (!first || !k || !U))) return fail(h, MPS_EINVAL, "bad gate list");
  std::vector<GateRef> gates;
  gates.reserve(count);
  size_t off = 0;
  const bool dd = h->prec == MPS_PREC_DD;
  for (int i = 0; i < count; ++i) {
    const double* lo = (U_lo && dd) ? U_lo + off : nullptr;
    int rc = validate_gate(h, first[i], k[i], U + off, lo, &h->err);
    if (rc) return rc;
    gates.push_back(GateRef{0, first[i], k[i], U + off, lo});
    off += (size_t)2 << (2 * k[i]);
  }
  if (!h->E->fuse) return run_state(h, gates);
  std::vector<double> hi, lo;
  return run_state(h, fuse_list(gates, dd, hi, lo));
}

int mps_apply_gate(mps_handle h, int first, int k, const double* U) {
  return mps_apply_gates(h, 1, &first, &k, U, nullptr);
}


// ------------------------------------------------------------------ non-adjacent gates
// A two-qubit gate on qubits q0, q1 (U's first index bit is q0).  Adjacent qubits
// take one U(4) update (U conjugated by SWAP when q0 > q1: an index permutation).
// Otherwise, with a < b the two qubits: SWAP updates carry qubit b's state from
// site b to site a + 2, one U(8) update on sites a..a+2 applies U to the outer
// sites (identity on the middle one), and SWAP updates carry it back.  All gates
// go to the scheduler as one list; each update is truncated like any other.
int mps_apply_gate2_dd(mps_handle h, int q0, int q1, const double* U_hi, const double* U_lo) {
  if (!h) return MPS_EINVAL;
  if (q0 < 0 || q1 < 0 || q0 >= h->n || q1 >= h->n || q0 == q1)
    return fail(h, MPS_EINVAL, "qubits must be distinct and in [0, n)");
  if (!U_hi) return fail(h, MPS_EINVAL, "null gate matrix");
  const bool dd = h->prec == MPS_PREC_DD;
  const double* lo_in = dd ? U_lo : nullptr;
  if (!finite_gate(2, U_hi) || (lo_in && !finite_gate(2, lo_in)))
    return fail(h, MPS_ENONFINITE, "gate matrix has a NaN or infinite entry");
  const int a = std::min(q0, q1), b = std::max(q0, q1);
  const int nswap = b - a >= 2 ? b - a - 2 : 0;
  // every matrix the list points at, hi then lo, allocated once (stable addresses)
  const size_t n4 = 32, n8 = 128;
  std::vector<double> hi(2 * nswap * n4 + n8 + n4), lo(hi.size(), 0.0);
  std::vector<GateRef> gates;
  double* sw_hi = hi.data();
  double* sw_lo = lo.data();
  swap_gate(sw_hi);  // one SWAP matrix serves every swap (its lo plane stays zero)
  double* g_hi = hi.data() + n4;
  double* g_lo = lo.data() + n4;
  if (b == a + 1) {
    if (q0 < q1) {
      std::memcpy(g_hi, U_hi, sizeof(double) * n4);
      if (lo_in) std::memcpy(g_lo, lo_in, sizeof(double) * n4);
    } else {
      reversed_gate(U_hi, g_hi);
      if (lo_in) reversed_gate(lo_in, g_lo);
    }
    gates.push_back(GateRef{0, a, 2, g_hi, dd ? g_lo : nullptr});
  } else {
    const int p0 = q0 == a ? 0 : 2, p1 = 2 - p0;
    outer_gate8(U_hi, p0, p1, g_hi);
    if (lo_in) outer_gate8(lo_in, p0, p1, g_lo);
    for (int p = b - 1; p >= a + 2; --p) gates.push_back(GateRef{0, p, 2, sw_hi, dd ? sw_lo : nullptr});
    gates.push_back(GateRef{0, a, 3, g_hi, dd ? g_lo : nullptr});
    for (int p = a + 2; p <= b - 1; ++p) gates.push_back(GateRef{0, p, 2, sw_hi, dd ? sw_lo : nullptr});
  }
  return run_state(h, gates);
}

int mps_apply_gate2(mps_handle h, int q0, int q1, const double* U) {
  return mps_apply_gate2_dd(h, q0, q1, U, nullptr);
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
  HIPCHK(h, hipStreamSynchronize(h->E->stream));
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
  Engine* E = h->E;
  const bool dd = h->prec == MPS_PREC_DD;
  const size_t nbits = align_up((size_t)count * h->n);
  const size_t o_ptr = nbits, o_ld = o_ptr + align_up(sizeof(void*) * 2 * h->n), o_out = o_ld + align_up(sizeof(int) * h->n);
  const size_t outb = (size_t)count * sizeof(double2) * (dd ? 2 : 1);
  int rc = ensure_small(E, o_out + align_up(outb), &h->err);
  if (rc) return rc;
  char* hs = E->h_stage;
  std::memcpy(hs, bits, (size_t)count * h->n);
  const double2** hp = (const double2**)(hs + o_ptr);
  for (int s = 0; s < h->n; ++s) {
    hp[s] = h->B[s];
    hp[h->n + s] = dd ? h->Blo[s] : nullptr;
  }
  int* hld = (int*)(hs + o_ld);
  for (int s = 0; s < h->n; ++s) hld[s] = h->capx[s + 1];
  HIPCHK(h, hipMemcpyAsync(E->d_small, hs, o_out, hipMemcpyHostToDevice, E->stream));
  mpsk::AmpArgs a{};
  a.B = (const double2* const*)(E->d_small + o_ptr);
  a.ld = (const int*)(E->d_small + o_ld);
  a.dimx = h->d_dimx;
  a.n = h->n;
  a.bits = (const unsigned char*)E->d_small;
  a.out = (double2*)(E->d_small + o_out);
  {
    Timed tm(E, 5);
    hipError_t e = dd ? mpsk::launch_amplitude_dd(a, (const double2* const*)(E->d_small + o_ptr) + h->n, count, E->stream)
                      : mpsk::launch_amplitude(a, count, E->stream);
    if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("amplitude: ") + hipGetErrorString(e));
  }
  HIPCHK(h, hipMemcpyAsync(hs + o_out, E->d_small + o_out, outb, hipMemcpyDeviceToHost, E->stream));
  HIPCHK(h, hipStreamSynchronize(E->stream));
  harvest_timing(E);
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

int mps_rdo_dd(mps_handle h, int count, const int* qubits, double* rho_hi, double* rho_lo) {
  if (!h || !qubits || !rho_hi) return MPS_EINVAL;
  const int n = h->n;
  if (count < 1 || count > 7) return fail(h, MPS_EINVAL, "rdo: count must be 1..7");
  std::vector<char> listed(n, 0);
  for (int t = 0; t < count; ++t) {
    if (qubits[t] < 0 || qubits[t] >= n) return fail(h, MPS_EINVAL, "rdo: qubit out of range");
    if (listed[qubits[t]]) return fail(h, MPS_EINVAL, "rdo: repeated qubit");
    listed[qubits[t]] = 1;
  }
  Engine* E = h->E;
  const bool dd = h->prec == MPS_PREC_DD;
  int s1 = 0;
  for (int s = 0; s < n; ++s)
    if (listed[s]) s1 = s;
  // sizes: left environments (D blocks of m x m), F, right environments, rho
  size_t maxE = 1, maxF = 1, maxR = 1;
  long D = 1;
  for (int s = 0; s <= s1; ++s) {
    const size_t ml = h->dimx[s], mr = h->dimx[s + 1];
    maxE = std::max(maxE, (size_t)D * ml * ml);
    maxF = std::max(maxF, (size_t)D * 2 * ml * mr);
    if (listed[s]) D *= 4;
    maxE = std::max(maxE, (size_t)D * mr * mr);
  }
  for (int s = n - 1; s > s1; --s) {
    const size_t ml = h->dimx[s], mr = h->dimx[s + 1];
    maxR = std::max(maxR, std::max(ml * ml, mr * mr));
    maxF = std::max(maxF, 2 * ml * mr);
  }
  maxR = std::max(maxR, (size_t)h->dimx[s1 + 1] * h->dimx[s1 + 1]);
  const size_t P = dd ? 2 : 1;
  const size_t oA = 0, oB = oA + align_up(maxE * 16) * P, oF = oB + align_up(maxE * 16) * P;
  const size_t oR1 = oF + align_up(maxF * 16) * P, oR2 = oR1 + align_up(maxR * 16) * P;
  const size_t oRho = oR2 + align_up(maxR * 16) * P, total = oRho + align_up((size_t)D * 16) * P;
  if ((double)total > E->ws_limit) return fail(h, MPS_ERANGE, "rdo: the contraction needs more than the workspace cap");
  int rc = ensure_ws(E, total, &h->err);
  if (rc) return rc;
  char* w = E->ws;
  auto hi = [&](size_t o) { return (double2*)(w + o); };
  auto lo = [&](size_t o, size_t elems) { return dd ? (double2*)(w + o + align_up(elems * 16)) : nullptr; };
  hipStream_t st = E->stream;
  hipError_t e = hipSuccess;
  {
    Timed tm(E, 7);
    // right environment R = 1 (1 x 1) at the right end, then sites n-1 .. s1+1
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    HIPCHK(h, hipMemcpyAsync(hi(oR1), &one, 16, hipMemcpyHostToDevice, st));
    if (dd) HIPCHK(h, hipMemcpyAsync(lo(oR1, maxR), &zero, 16, hipMemcpyHostToDevice, st));
    size_t rc_ = oR1, rn = oR2;
    for (int s = n - 1; s > s1 && e == hipSuccess; --s) {
      mpsk::RdoStep p{};
      p.B = h->B[s];
      p.Blo = dd ? h->Blo[s] : nullptr;
      p.ld = h->capx[s + 1];
      p.ml = h->dimx[s];
      p.mr = h->dimx[s + 1];
      p.E = hi(rc_); p.Elo = lo(rc_, maxR);
      p.F = hi(oF); p.Flo = lo(oF, maxF);
      p.En = hi(rn); p.Enlo = lo(rn, maxR);
      e = mpsk::launch_rdo_right(p, dd, st);
      std::swap(rc_, rn);
    }
    // left environment E = 1 at the left end, then sites 0 .. s1
    HIPCHK(h, hipMemcpyAsync(hi(oA), &one, 16, hipMemcpyHostToDevice, st));
    if (dd) HIPCHK(h, hipMemcpyAsync(lo(oA, maxE), &zero, 16, hipMemcpyHostToDevice, st));
    size_t ec = oA, en = oB;
    long Dc = 1;
    int l = 0;
    for (int s = 0; s <= s1 && e == hipSuccess; ++s) {
      mpsk::RdoStep p{};
      p.B = h->B[s];
      p.Blo = dd ? h->Blo[s] : nullptr;
      p.ld = h->capx[s + 1];
      p.ml = h->dimx[s];
      p.mr = h->dimx[s + 1];
      p.l = l;
      p.E = hi(ec); p.Elo = lo(ec, maxE);
      p.F = hi(oF); p.Flo = lo(oF, maxF);
      p.En = hi(en); p.Enlo = lo(en, maxE);
      e = mpsk::launch_rdo_left(p, (int)Dc, listed[s] != 0, dd, st);
      if (listed[s]) { Dc *= 4; ++l; }
      std::swap(ec, en);
    }
    if (e == hipSuccess) {
      mpsk::RdoStep p{};
      p.mr = h->dimx[s1 + 1];
      p.E = hi(ec); p.Elo = lo(ec, maxE);
      p.F = hi(rc_); p.Flo = lo(rc_, maxR);
      p.En = hi(oRho); p.Enlo = lo(oRho, (size_t)D);
      e = mpsk::launch_rdo_final(p, (int)Dc, dd, st);
    }
  }
  if (e != hipSuccess) return fail(h, MPS_EDEVICE, std::string("rdo: ") + hipGetErrorString(e));
  std::vector<double2> rh(D), rl(dd ? D : 0);
  HIPCHK(h, hipMemcpyAsync(rh.data(), hi(oRho), D * 16, hipMemcpyDeviceToHost, st));
  if (dd) HIPCHK(h, hipMemcpyAsync(rl.data(), lo(oRho, (size_t)D), D * 16, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  harvest_timing(E);
  // ascending-site order of the contraction -> the order the caller listed
  std::vector<int> sorted;
  for (int s = 0; s < n; ++s)
    if (listed[s]) sorted.push_back(s);
  std::vector<int> pos(count);
  for (int t = 0; t < count; ++t)
    pos[t] = (int)(std::find(sorted.begin(), sorted.end(), qubits[t]) - sorted.begin());
  const int dim = 1 << count;
  for (int r = 0; r < dim; ++r)
    for (int c = 0; c < dim; ++c) {
      int rs = 0, cs = 0;
      for (int t = 0; t < count; ++t) {
        rs |= ((r >> (count - 1 - t)) & 1) << (count - 1 - pos[t]);
        cs |= ((c >> (count - 1 - t)) & 1) << (count - 1 - pos[t]);
      }
      const size_t src = ((size_t)rs << count) + cs, dst = (size_t)r * dim + c;
      rho_hi[2 * dst] = rh[src].x;
      rho_hi[2 * dst + 1] = rh[src].y;
      if (rho_lo) {
        rho_lo[2 * dst] = dd ? rl[src].x : 0.0;
        rho_lo[2 * dst + 1] = dd ? rl[src].y : 0.0;
      }
    }
  return MPS_OK;
}

int mps_amplitudes_noalloc(mps_handle h, int count, const unsigned char* bits, double* out) {
  if (!h || count < 0 || (count > 0 && (!bits || !out))) return MPS_EINVAL;
  if (count == 0) return MPS_OK;
  for (long i = 0; i < (long)count * h->n; ++i)
    if (bits[i] > 1) return fail_na(h, MPS_EINVAL, "bits must be 0 or 1");
  for (int s = 0; s <= h->n; ++s)
    if (h->dimx[s] > 1024) return fail_na(h, MPS_ERANGE, "amplitude kernel supports bond dims up to 1024");
  Engine* E = h->E;
  const bool dd = h->prec == MPS_PREC_DD;
  const NoAllocLayout L = noalloc_layout(count, h->n, dd);
  if (L.end > kNoAllocScratch)
    return fail_na(h, MPS_ERANGE, "mps_amplitudes_noalloc: bits, tables and results exceed its 4 MiB scratch");
  hipError_t e = hipSuccess;
  char* base = (char*)scratch_on(E->device, &e);
  if (!base) return fail_na(h, MPS_EDEVICE, "scratch lookup", hipGetErrorString(e));
  // every table comes straight from the caller's or the handle's host memory (the
  // handle's vectors exist already); nothing is staged in pinned memory
  const size_t nb = (size_t)count * h->n;
  NACHK(h, hipMemcpyAsync(base, bits, nb, hipMemcpyHostToDevice, E->stream));
  NACHK(h, hipMemcpyAsync(base + L.ptr, h->B.data(), sizeof(void*) * h->n, hipMemcpyHostToDevice, E->stream));
  if (dd)
    NACHK(h, hipMemcpyAsync(base + L.ptr + sizeof(void*) * h->n, h->Blo.data(), sizeof(void*) * h->n,
                            hipMemcpyHostToDevice, E->stream));
  NACHK(h, hipMemcpyAsync(base + L.ld, h->capx.data() + 1, sizeof(int) * h->n, hipMemcpyHostToDevice, E->stream));
  mpsk::AmpArgs a{};
  a.B = (const double2* const*)(base + L.ptr);
  a.ld = (const int*)(base + L.ld);
  a.dimx = h->d_dimx;
  a.n = h->n;
  a.bits = (const unsigned char*)base;
  a.out = (double2*)(base + L.out);
  e = dd ? mpsk::launch_amplitude_dd(a, (const double2* const*)(base + L.ptr) + h->n, count, E->stream)
         : mpsk::launch_amplitude(a, count, E->stream);
  if (e != hipSuccess) return fail_na(h, MPS_EDEVICE, "amplitude", hipGetErrorString(e));
  NACHK(h, hipMemcpyAsync(out, base + L.out, (size_t)count * sizeof(double2) * (dd ? 2 : 1), hipMemcpyDeviceToHost,
                          E->stream));
  NACHK(h, hipStreamSynchronize(E->stream));
  return MPS_OK;
}

int mps_rdo(mps_handle h, int count, const int* qubits, double* rho) {
  if (!h || !rho) return MPS_EINVAL;
  if (h->prec != MPS_PREC_DD) return mps_rdo_dd(h, count, qubits, rho, nullptr);
  const int dim = (count >= 1 && count <= 7) ? 1 << count : 1;
  std::vector<double> lo((size_t)2 * dim * dim);
  int rc = mps_rdo_dd(h, count, qubits, rho, lo.data());
  if (rc) return rc;
  for (size_t i = 0; i < lo.size(); ++i) rho[i] += lo[i];
  return MPS_OK;
}

int mps_rdo_block(mps_handle h, int first, int last, double* rho) {
  if (!h) return MPS_EINVAL;
  if (first < 0 || last < first || last >= h->n) return fail(h, MPS_EINVAL, "rdo_block: need 0 <= first <= last < n");
  std::vector<int> q;
  for (int s = first; s <= last; ++s) q.push_back(s);
  return mps_rdo(h, (int)q.size(), q.data(), rho);
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
  HIPCHK(h, hipStreamSynchronize(h->E->stream));
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
  HIPCHK(h, hipStreamSynchronize(h->E->stream));
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

// ------------------------------------------------------------------ checkpoint image
// Layout (little-endian): magic "MPSCKPT1" | int32 version, n, chi_max, prec |
// double eps | int32 dims[n + 1] (padded to 8 bytes) | per bond 0..n-2 the Schmidt
// values (hi, then lo on dd) | per site the tensor [alpha][i][beta] as interleaved
// complex (hi, then lo on dd) | uint64 FNV-1a hash of everything before it.
namespace {

constexpr char kCkptMagic[8] = {'M', 'P', 'S', 'C', 'K', 'P', 'T', '1'};
constexpr int kCkptVersion = 1;

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

size_t ckpt_size(int n, int prec, const std::vector<int>& dims) {
  const size_t P = prec == MPS_PREC_DD ? 2 : 1;
  size_t b = 8 + 4 * 4 + 8 + ((size_t)(n + 1) * 4 + 7) / 8 * 8;
  for (int s = 1; s < n; ++s) b += P * 8 * (size_t)dims[s];
  for (int s = 0; s < n; ++s) b += P * 16 * (size_t)dims[s] * 2 * dims[s + 1];
  return b + 8;
}

}  // namespace

int mps_export(mps_handle h, void* buf, long cap, long* size) {
  if (!h || !size) return MPS_EINVAL;
  const size_t need = ckpt_size(h->n, h->prec, h->dimx);
  *size = (long)need;
  if (!buf) return MPS_OK;
  if (cap < (long)need) return fail(h, MPS_ERANGE, "checkpoint buffer too small");
  const bool dd = h->prec == MPS_PREC_DD;
  unsigned char* p = (unsigned char*)buf;
  size_t o = 0;
  auto put = [&](const void* src, size_t n) {
    std::memcpy(p + o, src, n);
    o += n;
  };
  put(kCkptMagic, 8);
  const int hdr[4] = {kCkptVersion, h->n, h->chi, h->prec};
  put(hdr, sizeof(hdr));
  put(&h->eps, 8);
  put(h->dimx.data(), sizeof(int) * (h->n + 1));
  while (o % 8) p[o++] = 0;
  for (int b = 0; b + 1 < h->n; ++b) {
    const int m = h->dimx[b + 1];
    int got = 0;
    double* hi = (double*)(p + o);
    double* lo = dd ? hi + m : nullptr;
    const int rc = mps_schmidt_dd(h, b, hi, lo, m, &got);
    if (rc) return rc;
    o += (dd ? 2 : 1) * 8 * (size_t)m;
  }
  for (int s = 0; s < h->n; ++s) {
    const long nd = (long)h->dimx[s] * 2 * h->dimx[s + 1] * 2;
    double* hi = (double*)(p + o);
    double* lo = dd ? hi + nd : nullptr;
    const int rc = mps_get_site(h, s, hi, lo, nd);
    if (rc) return rc;
    o += (dd ? 2 : 1) * 8 * (size_t)nd;
  }
  const uint64_t hsh = fnv1a(p, o);
  put(&hsh, 8);
  return o == need ? MPS_OK : fail(h, MPS_EDEVICE, "checkpoint size mismatch");
}

mps_handle mps_import(const void* buf, long size, void* hip_stream) {
  g_create_error.clear();
  const unsigned char* p = (const unsigned char*)buf;
  auto bad = [](const char* why) -> mps_handle {
    g_create_error = std::string("mps_import: ") + why;
    return nullptr;
  };
  if (!p || size < 48) return bad("no image");
  if (std::memcmp(p, kCkptMagic, 8) != 0) return bad("not a checkpoint image");
  int hdr[4];
  std::memcpy(hdr, p + 8, sizeof(hdr));
  if (hdr[0] != kCkptVersion) return bad("unknown image version");
  const int n = hdr[1], chi = hdr[2], prec = hdr[3];
  if (n < 1 || n > (1 << 20) || chi < 1 || (prec != MPS_PREC_FP64 && prec != MPS_PREC_DD)) return bad("bad header");
  double eps;
  std::memcpy(&eps, p + 24, 8);
  if ((size_t)size < 32 + ((size_t)(n + 1) * 4 + 7) / 8 * 8 + 8) return bad("image truncated");
  std::vector<int> dims(n + 1);
  std::memcpy(dims.data(), p + 32, sizeof(int) * (n + 1));
  if (dims[0] != 1 || dims[n] != 1) return bad("bad bond dims");
  for (int s = 1; s < n; ++s)
    if (dims[s] < 1 || dims[s] > chi) return bad("bad bond dims");
  const size_t need = ckpt_size(n, prec, dims);
  if ((size_t)size != need) return bad("image size does not match its header");
  uint64_t hsh;
  std::memcpy(&hsh, p + need - 8, 8);
  if (fnv1a(p, need - 8) != hsh) return bad("checksum mismatch");
  mps_handle h = mps_create_ex(n, chi, eps, prec, hip_stream);
  if (!h) return nullptr;
  const bool dd = prec == MPS_PREC_DD;
  const size_t P = dd ? 2 : 1;
  size_t o = 32 + ((size_t)(n + 1) * 4 + 7) / 8 * 8;
  // the image's arrays may be unaligned for double: copy them out
  std::vector<std::vector<double>> lh(n), ll(n), bh(n), bl(n);
  for (int b = 0; b + 1 < n; ++b) {
    const int m = dims[b + 1];
    lh[b].resize(m);
    std::memcpy(lh[b].data(), p + o, 8 * (size_t)m);
    if (dd) {
      ll[b].resize(m);
      std::memcpy(ll[b].data(), p + o + 8 * (size_t)m, 8 * (size_t)m);
    }
    o += P * 8 * (size_t)m;
  }
  for (int s = 0; s < n; ++s) {
    const size_t nd = (size_t)dims[s] * 2 * dims[s + 1] * 2;
    bh[s].resize(nd);
    std::memcpy(bh[s].data(), p + o, 8 * nd);
    if (dd) {
      bl[s].resize(nd);
      std::memcpy(bl[s].data(), p + o + 8 * nd, 8 * nd);
    }
    o += P * 8 * nd;
  }
  std::vector<const double*> Bp(n), Blp(n), lp(std::max(1, n - 1)), llp(std::max(1, n - 1));
  for (int s = 0; s < n; ++s) {
    Bp[s] = bh[s].data();
    Blp[s] = dd ? bl[s].data() : nullptr;
  }
  for (int b = 0; b + 1 < n; ++b) {
    lp[b] = lh[b].data();
    llp[b] = dd ? ll[b].data() : nullptr;
  }
  const int rc = mps_load(h, dims.data() + 1, Bp.data(), dd ? Blp.data() : nullptr, lp.data(),
                          dd ? llp.data() : nullptr);
  if (rc) {
    g_create_error = std::string("mps_import: ") + h->err;
    mps_destroy(h);
    return nullptr;
  }
  return h;
}

int mps_set_option(mps_handle h, int key, double value) {
  if (!h) return MPS_EINVAL;
  return set_option(h->E, h->prec, key, value, &h->err);
}

int mps_sync(mps_handle h) {
  if (!h) return MPS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->E->stream));
  harvest_timing(h->E);
  return MPS_OK;
}

int mps_kernel_time(mps_handle h, int cls, double* ms, long* launches, int reset) {
  if (!h || cls < 0 || cls >= 12) return MPS_EINVAL;
  Engine* E = h->E;
  HIPCHK(h, hipStreamSynchronize(E->stream));
  harvest_timing(E);
  if (cls == 11) {  // graph replays of Jacobi sweeps; *ms: graphs captured
    if (ms) *ms = (double)E->graphs_built;
    if (launches) *launches = E->graph_launches;
    if (reset) E->graph_launches = E->graphs_built = 0;
    return MPS_OK;
  }
  if (cls >= 8) {  // counters: update-sweeps of the FP64 Jacobi (8) and of the dd polish (9),
                   // splits finalised at a sweep limit (10)
    long& c = cls == 8 ? E->slot_sweeps : cls == 9 ? E->slot_sweeps_dd : E->noconv_updates;
    if (ms) *ms = 0.0;
    if (launches) *launches = c;
    if (reset) c = 0;
    return MPS_OK;
  }
  if (ms) *ms = E->tms[cls];
  if (launches) *launches = E->tcount[cls];
  if (reset) { E->tms[cls] = 0; E->tcount[cls] = 0; }
  return MPS_OK;
}

// ------------------------------------------------------------------ batches
mps_batch_handle mps_batch_create(int count, const int* n, const int* chi_max, const double* eps, int prec) {
  g_create_error.clear();
  if (count < 1 || !n || !chi_max || !eps || (prec != MPS_PREC_FP64 && prec != MPS_PREC_DD)) {
    g_create_error = "mps_batch_create: need count >= 1, per-circuit n, chi_max, eps and prec FP64 or DD";
    return nullptr;
  }
  for (int i = 0; i < count; ++i)
    if (n[i] < 1 || chi_max[i] < 1 || chi_max[i] > 2048 || !(eps[i] >= 0) || !std::isfinite(eps[i])) {
      g_create_error = "mps_batch_create: circuit " + std::to_string(i) +
                       " needs n >= 1, 1 <= chi_max <= 2048, finite eps >= 0";
      return nullptr;
    }
  mps_batch* b = new mps_batch();
  b->E = engine_new(prec, nullptr, &g_create_error);
  if (!b->E) {
    delete b;
    return nullptr;
  }
  b->E->batch = true;
  b->E->max_slots = 1024;
  size_t bytes = 0;
  for (int i = 0; i < count; ++i) {
    mps_state* h = new mps_state();
    state_shape(h, n[i], chi_max[i], eps[i], prec);
    h->E = b->E;
    h->batch = b;
    b->units.push_back(h);
    bytes += state_bytes(h, false);
    b->dims_total += n[i] + 1;
  }
  const size_t dims_bytes = align_up(sizeof(int) * b->dims_total);
  hipError_t e = hipMalloc((void**)&b->mem, bytes + dims_bytes);
  if (e == hipSuccess) e = hipMemsetAsync(b->mem, 0, bytes + dims_bytes, b->E->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("mps_batch_create: ") + hipGetErrorString(e);
    mps_batch_destroy(b);
    return nullptr;
  }
  char* p = b->mem;
  b->d_dims = (int*)(b->mem + bytes);
  int off = 0;
  for (mps_state* h : b->units) {
    p = state_carve(h, p, false);
    h->d_dimx = b->d_dims + off;
    off += h->n + 1;
  }
  if (set_product_states(b->E, b->units, b->d_dims, b->dims_total, &g_create_error)) {
    mps_batch_destroy(b);
    return nullptr;
  }
  return b;
}

int mps_batch_destroy(mps_batch_handle b) {
  if (!b) return MPS_EINVAL;
  engine_sync(b->E);
  for (mps_state* h : b->units) delete h;
  if (b->mem) (void)hipFree(b->mem);
  engine_free(b->E);
  delete b;
  return MPS_OK;
}

mps_handle mps_batch_get(mps_batch_handle b, int circuit) {
  if (!b || circuit < 0 || circuit >= (int)b->units.size()) return nullptr;
  return b->units[circuit];
}

int mps_batch_run(mps_batch_handle b, long ngates, const int* circuit, const int* first, const int* k,
                  const double* U, const double* U_lo) {
  if (!b) return MPS_EINVAL;
  if (ngates < 0 || (ngates > 0 && (!circuit || !first || !k || !U))) return fail(b, MPS_EINVAL, "bad gate list");
  const bool dd = b->E->prec == MPS_PREC_DD;
  std::vector<GateRef> gates;
  gates.reserve(ngates);
  size_t off = 0;
  for (long i = 0; i < ngates; ++i) {
    if (circuit[i] < 0 || circuit[i] >= (int)b->units.size())
      return fail(b, MPS_EINVAL, "gate " + std::to_string(i) + ": circuit index out of range");
    const double* lo = (U_lo && dd) ? U_lo + off : nullptr;
    int rc = validate_gate(b->units[circuit[i]], first[i], k[i], U + off, lo, &b->err);
    if (rc) {
      b->err = "gate " + std::to_string(i) + ": " + b->err;
      return rc;
    }
    gates.push_back(GateRef{circuit[i], first[i], k[i], U + off, lo});
    off += (size_t)2 << (2 * k[i]);
  }
  std::vector<int> dims_off;
  int o = 0;
  for (mps_state* h : b->units) {
    dims_off.push_back(o);
    o += h->n + 1;
  }
  if (!b->E->fuse) return run_sched(b->E, b->units, b->d_dims, b->dims_total, dims_off, gates, &b->err);
  std::vector<double> hi, lo;  // fusion circuit by circuit, the list's order kept
  return run_sched(b->E, b->units, b->d_dims, b->dims_total, dims_off, fuse_list(gates, dd, hi, lo), &b->err);
}

int mps_batch_set_option(mps_batch_handle b, int key, double value) {
  if (!b) return MPS_EINVAL;
  return set_option(b->E, b->E->prec, key, value, &b->err);
}

const char* mps_batch_last_error(mps_batch_handle b) { return b ? b->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
