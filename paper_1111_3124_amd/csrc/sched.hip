// The update scheduler: task workspace and descriptors, the Jacobi sweep plans,
// and the tick loop that runs a list of gates over one or more states.
#include "runtime.h"

namespace mpsrt {

constexpr int kQrMaxN = 1024;

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
  int passes = 0;  // dd refinement passes queued; `sweep` counts those whose outcome was read
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
// V's deferred rotations: two step parities of the pairs of the padded block count
size_t vp_pairs(int N) { return (size_t)((N + 7) / 8 + 2) / 2 * 2; }

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
  b += align_up(vp_pairs(N) * 256 * sizeof(double2)) + align_up(vp_pairs(N) * 17 * sizeof(int));  // deferred V
  b += align_up(((MN + mpsk::kFroChunk - 1) / mpsk::kFroChunk) * sizeof(double));  // ||theta_w||^2 partials
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
  t.VPR = (double2*)w;
  w += align_up(vp_pairs(t.N) * 256 * sizeof(double2));
  t.VPC = (int*)w;
  w += align_up(vp_pairs(t.N) * 17 * sizeof(int));
  t.frop = (double*)w;
  w += align_up(((MN + mpsk::kFroChunk - 1) / mpsk::kFroChunk) * sizeof(double));
  t.qr = 0;
  t.JW = t.thw;
  t.JR = t.JM;
  // V is accumulated where something reads it: the split's Z of a tall or square
  // theta, and the dd refinement; a wide FP64 theta takes Z from W's columns
  t.jvec = (dd || !t.tr) ? 1 : 0;
  t.JV = t.jvec ? t.V : nullptr;
  // the split's right factor: V, or for a wide theta W itself (its kept columns are
  // scaled to unit norm after the truncation)
  t.Z = t.tr ? t.thw : t.V;
  t.Z_lo = t.tr ? t.thw_lo : t.V_lo;
  t.flags = d_flags + 3 * slot;
  t.stats = d_stats + 8 * slot;
  t.fro2 = d_fro + slot;
}

// QR preconditioning of a Jacobi problem (theta_w P = Q R, Jacobi on R^H): two-site
// updates and either split of a three-site gate, tall or square thetas with 64 <= N
// and M <= 1024 (the panel kernel keeps at most two rows a thread), and for
// double-double only square ones (their refinement then runs on the transposed
// problem from the left singular vectors Q V).  FP64: the Jacobi's W is R^H in V's
// storage, V is not accumulated, Z is formed in theta_w's storage.
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
  bool defer_a = false, defer_b = false;  // fused steps with V's rotations deferred
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
        // (one-launch steps only: the two-launch form has no stamps)
        long long* pc =
            (P.phase && k == 0 && stp == nsteps / 2 && &g == &P.groups[0] && !g.split_a) ? P.phase : nullptr;
        if (g.na && stp < steps_of(g.mNa, g.bw)) {
          e = g.split_a
                  ? mpsk::launch_jacobi_split(dt, P.la[k] + g.oa, g.na, g.mNa, stp, E->tol_mult, E->max_inner,
                                              g.inner_few, st)
                  : mpsk::launch_jacobi_step(dt, P.la[k] + g.oa, g.na, g.mNa, g.bw, stp, E->tol_mult, E->max_inner,
                                             g.inner_few, g.defer_a, st, pc);
          if (e != hipSuccess) return e;
        }
        if (g.nb && stp < steps_of(g.mNb, g.bw)) {
          hipStream_t s2 = P.two ? E->stream2 : st;
          e = g.split_b ? mpsk::launch_jacobi_split(dt, P.lb[k] + g.ob, g.nb, g.mNb, stp, E->tol_mult, E->max_inner,
                                                    g.inner_few, s2)
                        : mpsk::launch_jacobi_step(dt, P.lb[k] + g.ob, g.nb, g.mNb, g.bw, stp, E->tol_mult,
                                                   E->max_inner, g.inner_few, g.defer_b, s2, nullptr);
          if (e != hipSuccess) return e;
        }
      }
    }
    if (k == P.K - 1) {  // V's rotations still deferred after the last step
      for (const SweepGroup& g : P.groups) {
        if (g.defer_a && (e = mpsk::launch_jacobi_vflush(dt, P.la[k] + g.oa, g.na, g.mNa, st)) != hipSuccess) return e;
        if (g.defer_b &&
            (e = mpsk::launch_jacobi_vflush(dt, P.lb[k] + g.ob, g.nb, g.mNb, P.two ? E->stream2 : st)) != hipSuccess)
          return e;
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
    for (long long v : {g.bw, g.inner_few, g.na, g.nb, g.oa, g.ob, g.mNa, g.mNb, (int)g.split_a, (int)g.split_b,
                        (int)g.defer_a, (int)g.defer_b})
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

// One run of the scheduler over a list of gates: the set-up sizes the slots, the
// workspace arena and the staging areas; each tick then admits gates, launches
// their theta (and QR factorisations), runs the sweeps of the iterating slots, reads
// the rotation flags and finalises converged slots (see the comment above Slot).
class Scheduler {
 public:
  Scheduler(Engine* E_, const std::vector<mps_state*>& U_, const int* d_dims_, int dims_total_,
            const std::vector<int>& dims_off_, const std::vector<GateRef>& gates_, std::string* err_)
      : E(E_), U(U_), d_dims(d_dims_), dims_total(dims_total_), dims_off(dims_off_), gates(gates_), err(err_) {}
  int run();

 private:
  // device lists: new2, new3, jacobi (two halves + order, for each of two sweeps), dd,
  // dd-enter, final, final3, mid, znorm, ref, polish, qr z, dd-enter QR tasks, and a
  // ring of kQrRing lists of QR factorisations in flight
  enum {
    LN2 = 0, LN3, LJ, LD, LENTER, LFIN, LFIN3, LMID, LZN, LR, LPOL, LJ2, LJO, LQZ, LQL, LJ_1, LJ2_1, LJO_1,
    LR_1, LEP0, LEP1, LQR0
  };
  static constexpr int kQrRing = 4;
  static constexpr int kLists = LQR0 + kQrRing;
  // dd refinement passes queued together (each after the first runs only if the one
  // before it corrected without converging), so that an update that needs two
  // passes reads both outcomes at one tick
  static constexpr int kRefChain = 2;
  // QR factorisations in flight on stream3, oldest first: completion event and the
  // slots waiting (state 6); polled at the end of each tick, so that a factorisation
  // longer than a sweep does not hold up the other updates' sweeps
  struct QrBatch {
    hipEvent_t ev;
    std::vector<int> slots;
  };

  int setup();
  int admit();            // 1. admission of queued gates
  int launch_admitted();  //    single-site gates; theta (and QR) of new slots
  int sweep();            // 2. dd passes and FP64 sweeps of the iterating slots
  int converge();         // 3. rotation flags read back, slot states advanced
  int finalise();         // 4. truncation and split of converged slots
  int finish();           // drain, timing, per-state diagnostics

  hipError_t fork_dd();
  hipError_t join_dd();
  void mark(int si) { dirty_lo = std::min(dirty_lo, si); dirty_hi = std::max(dirty_hi, si); }
  hipError_t upload_tasks();
  mpsk::Ent* upload_list(int li, const std::vector<mpsk::Ent>& ents);
  std::vector<mpsk::Ent> ents_of(const std::vector<int>& sl) const;
  hipError_t launch_jacobi(const std::vector<int>& jl, int K);
  hipError_t launch_passes(const std::vector<int>& sl, int l0, int l1);
  hipError_t qr_poll(bool block);
  int take_slot();
  void release_slot(int si);
  size_t ws_alloc(size_t need, size_t& off);
  char* hlist(int i) const { return E->h_stage + o_ents + i * list_bytes; }
  char* dlist(int i) const { return E->d_small + o_ents + i * list_bytes; }

  // the run's inputs
  Engine* E;
  const std::vector<mps_state*>& U;
  const int* d_dims;
  int dims_total;
  const std::vector<int>& dims_off;
  const std::vector<GateRef>& gates;
  std::string* err;
  // sizes and areas (setup)
  bool dd = false;
  int nu = 0, nsites = 0, S = 0;
  std::vector<int> site_base;
  std::vector<std::vector<int>> queue;  // per state: its gates in order
  size_t uniform = 0;                   // standalone engines: every slot's workspace
  size_t o_g1 = 0, o_ents = 0, list_bytes = 0;
  Task2* ht = nullptr;  // task descriptors: pinned staging and device copy
  Task2* dt = nullptr;
  int* d_flags = nullptr;
  int* hflags = nullptr;
  double* d_stats = nullptr;
  double* hstats = nullptr;
  double* d_fro = nullptr;
  int* hdims = nullptr;
  double2* hu8 = nullptr;
  double2* du8 = nullptr;
  // slots and gates
  std::vector<Slot> slot;
  std::vector<char> done, busy, claimed;
  std::vector<double> gstats;
  std::vector<int> gsweeps, gdd;
  std::vector<size_t> head;  // per state: first queue entry not yet admitted
  size_t remaining = 0;
  int status = MPS_OK;
  int rot0 = 0;  // first state scanned at admission (rotates for fairness)
  hipStream_t st = nullptr, sd = nullptr;
  bool sd_pending = false;
  int dirty_lo = 0, dirty_hi = -1;  // task descriptors changed since the last upload
  std::vector<int> free_list;       // free slot indices, lowest last
  std::vector<int> active;          // slots not free
  bool unsynced = false;            // async copies from the pinned staging may still be pending
  std::deque<QrBatch> qr_inflight;
  int qr_ring = 0;
  // the current tick
  std::vector<int> new2, new3;  // slots admitted (two-site, three-site first splits)
  std::vector<Task1> g1;        // single-site gates admitted
  long g1_maxel = 0;
  std::vector<int> jl, rl, dl;  // slots in FP64 sweeps, dd refinement, dd polish
  int K = 1;                    // FP64 sweeps this tick
  bool stamped = false;         // MPS_DEBUG_PHASES: this tick's launches stamped one step
};

int Scheduler::setup() {
  // a previous run that ended in an error may have left QR factorisations or dd work
  // queued: let them drain before any slot, list or workspace is reused
  HIPCHK(err, hipStreamSynchronize(E->stream3));
  HIPCHK(err, hipStreamSynchronize(E->stream4));
  dd = E->prec == MPS_PREC_DD;
  nu = (int)U.size();
  site_base.assign(nu + 1, 0);
  for (int u = 0; u < nu; ++u) site_base[u + 1] = site_base[u] + U[u]->n;
  nsites = site_base[nu];
  queue.assign(nu, {});
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
  S = std::max(n3 ? 2 : 1, std::min(std::min(E->max_slots, par), std::max(1, n2 + 2 * n3)));
  // standalone engines: every slot takes the same, largest workspace (no
  // fragmentation); batch engines: each update takes what its shape needs
  size_t arena_bytes;
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
  o_g1 = o_u8 + align_up(sizeof(double2) * 128 * S);
  o_ents = o_g1 + align_up(sizeof(Task1) * nsites);
  list_bytes = align_up(sizeof(mpsk::Ent) * S);
  rc = ensure_small(E, o_ents + kLists * list_bytes, err);
  if (rc) return rc;
  ht = (Task2*)(E->h_stage + o_tasks);
  dt = (Task2*)(E->d_small + o_tasks);
  d_flags = (int*)(E->d_small + o_flags);
  hflags = (int*)(E->h_stage + o_flags);
  d_stats = (double*)(E->d_small + o_stats);
  hstats = (double*)(E->h_stage + o_stats);
  d_fro = (double*)(E->d_small + o_fro);
  hdims = (int*)(E->h_stage + o_dims);
  hu8 = (double2*)(E->h_stage + o_u8);
  du8 = (double2*)(E->d_small + o_u8);
  slot.assign(S, Slot{});
  done.assign(gates.size(), 0);
  busy.assign(nsites, 0);
  claimed.assign(nsites, 0);
  gstats.assign(8 * gates.size(), 0.0);
  gsweeps.assign(gates.size(), 0);
  gdd.assign(gates.size(), 0);
  head.assign(nu, 0);
  remaining = gates.size();
  st = E->stream;
  // the dd work's stream; its launches follow everything queued on st so far (fork)
  // and st waits for them before reading flags back (join)
  sd = (dd && E->dd_stream) ? E->stream4 : st;
  dirty_lo = S;
  dirty_hi = -1;
  for (int si = S - 1; si >= 0; --si) free_list.push_back(si);
  return MPS_OK;
}

hipError_t Scheduler::fork_dd() {
  if (sd == st) return hipSuccess;
  hipError_t ee = hipEventRecord(E->ev_dd_fork, st);
  if (ee == hipSuccess) ee = hipStreamWaitEvent(sd, E->ev_dd_fork, 0);
  sd_pending = true;
  return ee;
}

hipError_t Scheduler::join_dd() {
  if (!sd_pending) return hipSuccess;
  sd_pending = false;
  hipError_t ee = hipEventRecord(E->ev_dd_join, sd);
  if (ee == hipSuccess) ee = hipStreamWaitEvent(st, E->ev_dd_join, 0);
  return ee;
}

hipError_t Scheduler::upload_tasks() {
  if (dirty_hi < dirty_lo) return hipSuccess;
  hipError_t ee = hipMemcpyAsync(dt + dirty_lo, ht + dirty_lo, sizeof(Task2) * (dirty_hi - dirty_lo + 1),
                                 hipMemcpyHostToDevice, st);
  dirty_lo = S;
  dirty_hi = -1;
  return ee;
}

mpsk::Ent* Scheduler::upload_list(int li, const std::vector<mpsk::Ent>& ents) {
  mpsk::Ent* hl = (mpsk::Ent*)hlist(li);
  for (size_t i = 0; i < ents.size(); ++i) hl[i] = ents[i];
  hipError_t ee = hipMemcpyAsync(dlist(li), hl, sizeof(mpsk::Ent) * ents.size(), hipMemcpyHostToDevice, st);
  return ee == hipSuccess ? (mpsk::Ent*)dlist(li) : nullptr;
}

std::vector<mpsk::Ent> Scheduler::ents_of(const std::vector<int>& sl) const {
  std::vector<mpsk::Ent> v;
  v.reserve(sl.size());
  for (int si : sl) v.push_back(mpsk::Ent{si, slot[si].sweep});
  return v;
}

// up to kRefChain dd refinement passes for each slot of `sl` (within the pass
// limit) on the dd stream, the k-th pass of the chain from the list l0 (k = 0) or
// l1 (k = 1)
hipError_t Scheduler::launch_passes(const std::vector<int>& sl, int l0, int l1) {
  const int lists[kRefChain] = {l0, l1};
  for (int k = 0; k < kRefChain; ++k) {
    std::vector<mpsk::Ent> ents;
    int mM = 0, mN = 0;
    for (int si : sl)
      if (slot[si].passes + k < E->max_ref_passes) {
        ents.push_back(mpsk::Ent{si, slot[si].passes + k});
        mM = std::max(mM, slot[si].JM);
        mN = std::max(mN, slot[si].N);
      }
    if (ents.empty()) break;
    mpsk::Ent* el = upload_list(lists[k], ents);
    if (!el) return hipErrorInvalidValue;
    Timed tm(E, 6, 1, sd);
    const hipError_t e = mpsk::launch_ddref_pass(dt, el, (int)ents.size(), mM, mN, E->tol_mult, sd);
    if (e != hipSuccess) return e;
  }
  for (int si : sl) slot[si].passes = std::min(slot[si].passes + kRefChain, E->max_ref_passes);
  return hipSuccess;
}

// the FP64 sweeps of the iterating slots `jl` (K of them), as stream launches or
// as a replayed graph
hipError_t Scheduler::launch_jacobi(const std::vector<int>& jl, int K) {
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
    auto any_v = [&](const std::vector<int>& v) {
      for (int si : v)
        if (ht[si].jvec) return true;
      return false;
    };
    // the one-launch step of block width 8 defers V's rotations by a step (its launches
    // then carry the V blocks)
    g.defer_a = g.bw == 8 && !g.split_a && any_v(ga[gi]);
    g.defer_b = g.bw == 8 && !g.split_b && any_v(gb[gi]);
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
  // (the stamps come from a one-launch step of the first group's half a)
  stamped = E->d_phase && !P.groups.empty() && P.groups[0].na && !P.groups[0].split_a;
  Timed tm(E, 1, K * plan_steps(P));
  if (E->graphs_on && !E->d_phase) return launch_sweep_graph(E, dt, P, st);
  return enqueue_sweeps(E, dt, P, st);
}

int Scheduler::take_slot() {
  const int si = free_list.back();
  free_list.pop_back();
  return si;
}

void Scheduler::release_slot(int si) {
  if (slot[si].ws_len) E->arena.release(slot[si].ws_off, slot[si].ws_len);
  slot[si] = Slot{};
  free_list.push_back(si);
}

size_t Scheduler::ws_alloc(size_t need, size_t& off) {
  const size_t len = align_up(uniform ? uniform : need);
  off = E->arena.alloc(len);
  return off == SIZE_MAX ? (size_t)0 : len;
}

hipError_t Scheduler::qr_poll(bool block) {
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
}

int Scheduler::admit() {
  // ---- 1. admission
  new2.clear();
  new3.clear();
  g1.clear();
  g1_maxel = 0;
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
          if (cfg.qr) qr_select(dd, t);  // two-site updates and first splits of three-site gates
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
  return MPS_OK;
}

int Scheduler::launch_admitted() {
  hipError_t e;
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
      if (e == hipSuccess) {
        long mn = 0;
        for (int si : nl) mn = std::max(mn, (long)slot[si].M * slot[si].Nt);
        e = mpsk::launch_fro(dt, el, (int)nl.size(), mn, st);
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
  return MPS_OK;
}

int Scheduler::sweep() {
  hipError_t e;
  // dd refinement passes and polish sweeps first, on the dd stream, so that they
  // overlap the FP64 sweeps launched below
  // (slots whose queued passes have not been read yet get no new ones)
  std::vector<int> rq;
  for (int si : rl)
    if (slot[si].passes == slot[si].sweep) rq.push_back(si);
  if (!rq.empty() || !dl.empty()) {
    mpsk::Ent* eld = dl.empty() ? nullptr : upload_list(LD, ents_of(dl));
    if (!dl.empty() && !eld) return fail(err, MPS_EDEVICE, "list upload failed");
    HIPCHK(err, fork_dd());
    if (!rq.empty()) {
      e = launch_passes(rq, LR, LR_1);
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
  K = 1;  // sweeps this tick
  stamped = false;
  if (!jl.empty()) {
    K = std::max(1, std::min(2, E->tick_sweeps));
    for (int si : jl) K = std::min(K, E->max_sweeps - slot[si].sweep);
    K = std::max(K, 1);
    HIPCHK(err, launch_jacobi(jl, K));
  }
  return MPS_OK;
}

int Scheduler::converge() {
  hipError_t e;
  // finished QR factorisations: their slots start iterating at the next tick; when
  // this tick has no sweep work at all, wait for the oldest
  HIPCHK(err, qr_poll(jl.empty() && rl.empty() && dl.empty()));
  // ---- 3. convergence
  HIPCHK(err, join_dd());
  if (!jl.empty() || !rl.empty() || !dl.empty()) {
    HIPCHK(err, hipMemcpyAsync(hflags, d_flags, sizeof(int) * 3 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(err, hipStreamSynchronize(st));
    unsynced = false;
    if (stamped && !jl.empty()) {
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
        sl.passes = 0;
      } else {
        sl.conv = sl.fp64_conv;
        sl.state = 3;
      }
    }
  }
  std::vector<int> to_polish;
  for (int si : rl) {
    Slot& sl = slot[si];
    // the queued passes in order, up to the first that converged or was void (the
    // ones after it changed nothing)
    while (sl.sweep < sl.passes) {
      const int code = hflags[3 * si + sl.sweep % 3];
      ++sl.sweep;
      ++E->slot_sweeps_dd;
      if (code == 0) {
        sl.dd_sweeps = sl.sweep;
        sl.conv = true;
        sl.state = 3;
        break;
      }
      if ((code & 2) || sl.sweep >= E->max_ref_passes) {
        sl.dd_sweeps = sl.sweep;
        sl.state = 4;
        sl.sweep = 0;
        to_polish.push_back(si);
        break;
      }
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
    {
      Timed tm(E, 6, 1, sd);
      e = mpsk::launch_dd_enter(dt, el, (int)enter.size(), mM, mN, sd);
      if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("dd enter: ") + hipGetErrorString(e));
    }
    // the first refinement passes follow the promotion at once; their outcome is
    // read at the next tick
    std::vector<int> rq;
    for (int si : enter)
      if (slot[si].state == 2) rq.push_back(si);
    if (!rq.empty()) {
      e = launch_passes(rq, LEP0, LEP1);
      if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("dd refinement: ") + hipGetErrorString(e));
    }
  }
  return MPS_OK;
}

int Scheduler::finalise() {
  hipError_t e;
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
    std::vector<int> newB, qr2;
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
      if (cfg.qr) qr_select(dd, tb);
      if (tb.qr) {  // the second split's theta is factorised too, on stream3 after k_mid3
        sbl.state = 6;
        qr2.push_back(sb);
      }
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
        if (e == hipSuccess) {
          long mn = 0;
          for (int sb : newB) mn = std::max(mn, (long)ht[sb].M * ht[sb].Nt);
          e = mpsk::launch_fro(dt, eb, (int)newB.size(), mn, st);
        }
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("mid: ") + hipGetErrorString(e));
      }
      if (!qr2.empty()) {
        int qM = 0, qN = 0;
        for (int sb : qr2) {
          qM = std::max(qM, ht[sb].M);
          qN = std::max(qN, ht[sb].N);
        }
        if ((int)qr_inflight.size() >= kQrRing) HIPCHK(err, qr_poll(true));  // frees the oldest ring slot
        mpsk::Ent* eq = upload_list(LQR0 + qr_ring, ents_of(qr2));
        if (!eq) return fail(err, MPS_EDEVICE, "list upload failed");
        qr_ring = (qr_ring + 1) % kQrRing;
        HIPCHK(err, hipEventRecord(E->ev_qr, st));
        HIPCHK(err, hipStreamWaitEvent(E->stream3, E->ev_qr, 0));
        e = mpsk::launch_qr_factor(dt, eq, (int)qr2.size(), qM, qN, E->stream3);
        if (e != hipSuccess) return fail(err, MPS_EDEVICE, std::string("qr: ") + hipGetErrorString(e));
        hipEvent_t done = ev_get(E);
        if (!done) return fail(err, MPS_EDEVICE, "event creation failed");
        HIPCHK(err, hipEventRecord(done, E->stream3));
        qr_inflight.push_back(QrBatch{done, qr2});
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
  return MPS_OK;
}

int Scheduler::finish() {
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

int Scheduler::run() {
  if (gates.empty()) return MPS_OK;
  int rc = setup();
  if (rc) return rc;
  while (true) {
    // the staging buffers are rewritten below: wait for copies a previous tick left
    if (unsynced) {
      HIPCHK(err, hipStreamSynchronize(st));
      unsynced = false;
    }
    if ((rc = admit()) || (rc = launch_admitted())) return rc;
    // one sweep for every iterating slot (QR-pending slots wait)
    jl.clear();
    rl.clear();
    dl.clear();
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
    if ((rc = sweep()) || (rc = converge()) || (rc = finalise())) return rc;
  }
  return finish();
}

int run_sched(Engine* E, const std::vector<mps_state*>& U, const int* d_dims, int dims_total,
              const std::vector<int>& dims_off, const std::vector<GateRef>& gates, std::string* err) {
  Scheduler s(E, U, d_dims, dims_total, dims_off, gates, err);
  return s.run();
}

int run_state(mps_state* h, const std::vector<GateRef>& gates) {
  return run_sched(h->E, {h}, h->d_dimx, h->n + 1, {0}, gates, &h->err);
}


}  // namespace mpsrt
