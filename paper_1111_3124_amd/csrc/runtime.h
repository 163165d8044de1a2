// Internal interface of the host runtime (not installed): engines, states and
// batches, the shared error helpers, and the entry points of the scheduler
// (sched.hip) and of the engine code (engine.hip) used by the C ABI (runtime.hip).
//
// An engine owns everything a run of the scheduler needs besides the states: one
// standalone handle owns one engine; a batch owns one engine shared by all its
// states, so the updates of every circuit of the batch run in the same launches.
// Bond dimensions live in device tables written by the truncation kernel; the
// host mirrors them after each finalisation (one small device-to-host copy), so
// that every launch is sized to the live shapes.
#pragma once

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

namespace mpsrt {

using mpsk::Task1;
using mpsk::Task2;

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

// step configuration of a Jacobi problem (block width, inner sweeps with few
// blocks, QR preconditioning)
struct StepCfg {
  int bw, inner_few, qr;
};

// one gate of a scheduler run: the state it acts on (index in the run's state list)
struct GateRef {
  int unit;  // index of the state in the run's state list
  int first, k;
  const double* U;
  const double* Ulo;
};

}  // namespace mpsrt

struct mps_state {
  int n = 0, chi = 0, prec = MPS_PREC_FP64;
  double eps = 0.0;
  mpsrt::Engine* E = nullptr;
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
  mpsrt::Engine* E = nullptr;
  std::vector<mps_state*> units;
  char* mem = nullptr;  // one device block for every state
  int* d_dims = nullptr;  // all bond-dimension tables, back to back
  int dims_total = 0;
  std::string err;
};

namespace mpsrt {

inline int fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}
inline int fail(mps_state* h, int code, const std::string& msg) { return fail(h ? &h->err : nullptr, code, msg); }
inline int fail(mps_batch* b, int code, const std::string& msg) { return fail(b ? &b->err : nullptr, code, msg); }

#define HIPCHK(h, call)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(h, e_ == hipErrorOutOfMemory ? MPS_ENOMEM : MPS_EDEVICE,                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                          \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// engine.hip
std::string tuning_key(int device);
std::vector<TuneEntry> tuning_for(int device);
StepCfg step_cfg(const Engine* E, int N);
Engine* engine_new(int prec, void* hip_stream, std::string* err);
void engine_sync(Engine* E);
void engine_free(Engine* E);
hipEvent_t ev_get(Engine* E);
void harvest_timing(Engine* E);
int ensure_ws(Engine* E, size_t bytes, std::string* err);
int ensure_small(Engine* E, size_t bytes, std::string* err);
int set_option(Engine* E, int prec, int key, double value, std::string* err);

// sched.hip
// Runs `gates` on the states `U` of engine E.  d_dims / dims_total: one device range
// covering every state's bond-dimension table; dims_off[u] = offset of state u's.
int run_sched(Engine* E, const std::vector<mps_state*>& U, const int* d_dims, int dims_total,
              const std::vector<int>& dims_off, const std::vector<GateRef>& gates, std::string* err);
int run_state(mps_state* h, const std::vector<GateRef>& gates);

// HIP events bracketing a kernel class's launches (when the engine's timing is on)
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

}  // namespace mpsrt
