// The C ABI of include/mps.h: states and batches (device memory, product states,
// loading, checkpoints), gate validation and fusion, readout (Schmidt values,
// amplitudes, reduced density operators) and options; updates go to the scheduler.
#include "runtime.h"

using namespace mpsrt;

namespace {

thread_local std::string g_create_error;

int bond_capacity(int n, int chi, int b) {
  // min(chi, 2^{b+1}, 2^{n-1-b})
  long c = chi;
  int l = b + 1, r = n - 1 - b;
  if (l < 31) c = std::min(c, 1L << l);
  if (r < 31) c = std::min(c, 1L << r);
  return (int)c;
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

