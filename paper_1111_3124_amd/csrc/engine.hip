// Engines (streams, workspace arena, pinned staging, event timing), the tuning
// table of per-size Jacobi step configurations, and the engine options.
#include "runtime.h"

namespace mpsrt {

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
StepCfg step_cfg(const Engine* E, int N) {
  if (E->tuned)
    for (const TuneEntry& t : E->tune)
      if (t.prec == E->prec && N <= t.nmax) return StepCfg{t.bw, t.inner_few, t.qr};
  return StepCfg{E->block_width, E->max_inner_few, E->qr ? 1 : 0};
}
// ------------------------------------------------------------------ engines
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

}  // namespace mpsrt
