/* mps.h -- C ABI of the MI355X matrix-product-state gate-update library.
 *
 * The library keeps an n-qubit pure state in the matrix-product form of the
 * paper's Section 3.1, Eq. (1), and applies quantum gates to it the way that
 * section describes: a gate on qubits s (and s+1, s+2) updates only the tensors
 * of those sites and the Schmidt coefficients between them (Eq. (2)); small
 * Schmidt coefficients are truncated away.
 *
 * Representation (device memory, owned by the handle):
 *   - Site s holds B_s[alpha][i][beta] = Q_s(i, alpha, beta) V_s(beta): the paper's
 *     Q_s with the Schmidt coefficients of its right bond absorbed, so that every
 *     B_s is right-canonical and no step divides by a Schmidt value.
 *   - Bond s (between sites s and s+1, s = 0..n-2) holds m_s and the Schmidt
 *     coefficients V_s(0..m_s-1) in descending order, with sum V_s^2 = 1.
 *   The amplitude c_{i0..i(n-1)} of Eq. (1) is B_0[i0] B_1[i1] ... B_{n-1}[i(n-1)].
 *
 * Conventions:
 *   - Qubit 0 is the leftmost qubit of |i_0 ... i_{n-1}>.
 *   - A k-qubit gate U (k = 1, 2, 3) acts on sites first..first+k-1; it is a
 *     2^k x 2^k complex matrix, row-major, U[r][c] = <r|U|c>, with basis index
 *     r = sum_t i_{first+t} 2^{k-1-t} (the first site is the most significant bit).
 *     It is passed as 2 * 4^k doubles, complex interleaved (re, im).
 *   - Truncation after each split: with the singular values sigma_j sorted
 *     descending and W = sum_j sigma_j^2, the kept count is
 *       k = min(chi_max, k_eps, rank),
 *     k_eps the smallest k >= 1 with sum_{j>=k} sigma_j^2 <= eps * W, and rank the
 *     number of sigma_j above the precision's noise floor relative to sigma_0.
 *     The kept values are renormalised: V_s = sigma_j / sqrt(sum_{j<k} sigma_j^2).
 *   - A three-qubit gate splits left first (s | s+1 s+2), then (s+1 | s+2).
 *   - Status: every int-returning call returns MPS_OK (0) or a negative MPS_E*
 *     code; mps_last_error() gives a message.  No exception crosses the ABI.
 *   - Ownership: the caller owns every host buffer passed in or out; the library
 *     copies inputs before returning.  The handle owns all device memory.
 *   - Synchronisation: gate application is queued on the handle's HIP stream.
 *     The library reads back each new bond dimension once its update has
 *     converged (it sizes later launches), so a gate call returns after the
 *     device has finished all but the final writes of its last update; every
 *     call that returns host data synchronises.
 *   - Threads: one thread at a time per handle.
 */
#ifndef MPS_H_
#define MPS_H_

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_state* mps_handle;

enum mps_status {
  MPS_OK = 0,
  MPS_EINVAL = -1,     /* bad argument (site out of range, k not in {1,2,3}, null buffer) */
  MPS_ERANGE = -2,     /* size beyond a documented limit or a caller buffer too small   */
  MPS_ENOMEM = -3,     /* device allocation failed                                      */
  MPS_EDEVICE = -4,    /* a HIP runtime call failed                                     */
  MPS_ENOCONV = -5,    /* the Jacobi iteration hit its sweep limit (state still updated) */
  MPS_ENONFINITE = -6, /* a gate entry is NaN or infinite                               */
  MPS_ESTATE = -7      /* operation not valid for this handle (e.g. dd call on FP64)    */
};

enum mps_precision {
  MPS_PREC_FP64 = 0,   /* binary64 tensors and arithmetic                               */
  MPS_PREC_DD = 1      /* double-double (hi + lo) tensors; FP64 SVD refined in dd       */
};

enum mps_option {
  MPS_OPT_MAX_SWEEPS = 1,     /* Jacobi sweep limit (default 40 FP64, 16 dd polish)      */
  MPS_OPT_JACOBI_TOL = 2,     /* relative off-diagonal tolerance multiplier (default 1)  */
  MPS_OPT_KERNEL_TIMING = 3,  /* 1: time every kernel class with HIP events (see below)  */
  MPS_OPT_RANK_FLOOR = 4,     /* relative rank floor (default 2^-44 FP64, 2^-96 dd)       */
  MPS_OPT_BLOCK_WIDTH = 5,    /* Jacobi column block width: 4, 8 (default) or 16          */
  MPS_OPT_MAX_INNER = 6,      /* inner sweeps per block pair, tasks with >= 16 blocks (1)  */
  MPS_OPT_MAX_SLOTS = 7,      /* updates in flight at once (default 32; batches 1024)     */
  MPS_OPT_WORKSPACE_MB = 8,   /* batches: cap of the update workspace, MiB (16384)        */
  MPS_OPT_DD_REFINE = 9,      /* dd: 1 (default) simultaneous first-order corrections,
                                 then the pairwise polish only where those do not apply;
                                 0: the pairwise dd Jacobi polish alone                  */
  MPS_OPT_JACOBI_STREAMS = 10,/* 2 (default): the FP64 Jacobi steps of concurrent updates
                                 run as two launch sequences on two internal streams,
                                 joined into the handle's stream; 1: one sequence        */
  MPS_OPT_FUSE = 11,          /* 1 (default): mps_apply_gates and mps_batch_run multiply
                                 a single-site gate into the latest earlier gate
                                 touching its site, and latest earlier single-site
                                 gates into a later gate on their sites (products in
                                 double-double; the same state up to rounding, since a
                                 one-site unitary keeps every cut's Schmidt values);
                                 multi-site gates are never merged.  0: off             */
  MPS_OPT_QR = 12             /* 1 (default): Jacobi problems (two-site updates and both
                                 splits of three-site gates) with 64 <= N <= M <= 1024
                                 (dd: square only) are preconditioned by a Householder
                                 QR of theta_w with its columns in norm order, and the
                                 Jacobi runs on R^H (fewer sweeps); a wide theta, run
                                 as theta_w^H, is not; 0: the Jacobi runs on theta_w    */,
  MPS_OPT_STEP_SPLIT = 13     /* block width 8: a Jacobi step launch that serves at most
                                 this many updates (default 4; 0: none) runs as two
                                 launches (partial Grams, then rotations and updates) of
                                 two 256-thread blocks a column-block pair, for more
                                 parallelism when few updates are in flight             */,
  MPS_OPT_DD_STREAM = 14      /* 1 (default): dd refinement passes, dd polish sweeps and
                                 the dd promotion of converged updates run on a stream of
                                 their own, overlapping the FP64 sweeps of the others;
                                 0: on the handle's stream                              */,
  MPS_OPT_MAX_INNER_FEW = 15  /* inner sweeps per block pair for tasks with fewer than 16
                                 column blocks (default 1 FP64, 12 dd; up to that many
                                 sweeps over all the pair's column pairs, ending early
                                 once one rotates nothing)                              */,
  MPS_OPT_TICK_SWEEPS = 16    /* FP64 Jacobi sweeps launched per scheduler tick, 1 or 2
                                 (default 2).  Convergence is tested on the device: an
                                 update whose last sweep rotated nothing skips every
                                 later one, so results do not depend on this value; the
                                 host reads the rotation flags once per tick           */,
  MPS_OPT_GRAPH = 17          /* 1: each tick's Jacobi sweeps (order kernels, step
                                 launches on both streams) are replayed from a HIP graph
                                 captured once per launch shape and kept by the engine;
                                 0 (default): launched one by one.  Same results      */
};

/* Diagnostics of the most recent split (the last one of a three-qubit gate). */
struct mps_update_stats {
  double W;        /* total weight sum sigma_j^2 before truncation                     */
  double w;        /* discarded weight, relative: sum_{j>=k} sigma_j^2 / W              */
  double gap;      /* (sigma_{k-1} - sigma_k) / sigma_0 when a non-zero value was cut, else +inf */
  double epsdist;  /* relative distance of the eps decision from its boundary, +inf if eps = 0 */
  int k;           /* kept count                                                      */
  int rank;        /* values above the rank floor                                     */
  int sweeps;      /* most FP64 Jacobi sweeps any update of the last call took          */
  int splits;      /* number of splits in the last gate (0, 1 or 2)                    */
  int dd_sweeps;   /* most dd polish sweeps any update of the last call took (dd)       */
  int reserved;
};

/* --- lifetime ------------------------------------------------------------------- */

/* Create an n-qubit state |0...0> (paper, Section 3.2: "mps M(n)"): all m_s = 1,
 * V_s = [1], B_s[0][0][0] = 1.  FP64 precision, the library's own stream.
 * n >= 1, chi_max >= 1, eps >= 0.  Returns NULL on error (see mps_last_error(NULL)). */
mps_handle mps_create(int n, int chi_max, double eps);

/* As mps_create with a precision (enum mps_precision) and an optional HIP stream
 * (hipStream_t passed as void*; NULL = a stream the handle creates and owns). */
mps_handle mps_create_ex(int n, int chi_max, double eps, int prec, void* hip_stream);

int mps_destroy(mps_handle h);

/* --- gates (Section 3.1: U(2), U(4), U(8) are elementary) ----------------------- */

/* Apply U (2 * 4^k doubles, see Conventions) to sites first..first+k-1.
 * k = 1: B_first <- (U (x) 1) B_first; no SVD, Schmidt values unchanged.
 * k = 2: theta = B_s B_{s+1} mixed by U, SVD of diag(V_{s-1}) theta, truncation,
 *        split into B_s, V_s, B_{s+1} (Section 3.1; Vidal's update).
 * k = 3: theta = B_s B_{s+1} B_{s+2} mixed by U (8 x 8), SVD of the
 *        (2 m_{s-1}) x (4 m_{s+2}) matrix diag(V_{s-1}) theta, truncation, split
 *        into B_s, V_s and the right factor; the right factor weighted by V_s
 *        is reshaped to (2 m_s) x (2 m_{s+2}) and split again into B_{s+1},
 *        V_{s+1}, B_{s+2}.  mps_stats then describes the second split.
 * Errors: MPS_EINVAL (first < 0, first + k > n, k not 1..3, U NULL),
 * MPS_ENONFINITE, MPS_ENOCONV, MPS_EDEVICE, MPS_ENOMEM. */
int mps_apply_gate(mps_handle h, int first, int k, const double* U);

/* Double-double gate: U = U_hi + U_lo exactly (same layout each).  On an FP64
 * handle U_lo is ignored. */
int mps_apply_gate_dd(mps_handle h, int first, int k, const double* U_hi, const double* U_lo);

/* Two-qubit gate on any two distinct qubits q0, q1 (the paper's applyU(U, q0, q1);
 * its Section 3.2 example applies CNOT to qubits 0 and 2).  U is 4 x 4 (2 * 16
 * doubles, see Conventions); the first (most significant) bit of its index belongs
 * to q0.  Adjacent qubits: one U(4) update on min(q0, q1), with U's qubits
 * exchanged when q0 > q1.  Otherwise, with a = min(q0, q1), b = max(q0, q1): SWAP
 * updates on sites (b-1, b), (b-2, b-1), ..., (a+2, a+3) carry qubit b's state to
 * site a+2, one U(8) update on sites a..a+2 applies U to the two outer sites (the
 * identity on site a+1), and SWAP updates on (a+2, a+3), ..., (b-1, b) carry it
 * back: 2 (b - a - 2) + 1 updates, each truncated like any other.  The input is
 * copied before return.  Errors: MPS_EINVAL (q0 == q1, a qubit outside [0, n),
 * U NULL), MPS_ENONFINITE, and those of mps_apply_gates. */
int mps_apply_gate2(mps_handle h, int q0, int q1, const double* U);

/* Double-double form of mps_apply_gate2 (U = U_hi + U_lo); U_lo ignored on FP64. */
int mps_apply_gate2_dd(mps_handle h, int q0, int q1, const double* U_hi, const double* U_lo);

/* Apply `count` gates in order.  The library's scheduler admits a gate as soon as
 * none of its sites is held by an unfinished update and no earlier, still
 * waiting gate touches them; admitted updates iterate together, one batched
 * launch per kernel and Jacobi step for all of them, and each finishes as soon
 * as its own SVD has converged.  Only gates on disjoint sites ever run at the
 * same time and gates on shared sites keep their order, so the result equals
 * applying the gates one by one.  first[i], k[i]; U packed back to back
 * (2 * 4^k[i] doubles each); U_lo NULL or same packing.  Every gate is checked
 * before any runs: an invalid one (MPS_EINVAL, MPS_ENONFINITE) applies none of
 * the list.  MPS_ENOCONV (some update hit the sweep limit; its result is still
 * used) is reported after all gates ran; MPS_EDEVICE leaves the state undefined. */
int mps_apply_gates(mps_handle h, int count, const int* first, const int* k,
                    const double* U, const double* U_lo);

/* --- readout --------------------------------------------------------------------- */

/* Bond dimension m_bond, bond in [0, n-2]. */
int mps_bond_dim(mps_handle h, int bond, int* m);

/* Schmidt coefficients V_bond (Eq. (2)), descending, into lam[0..m-1]; cap is the
 * capacity of lam; *m receives m_bond.  MPS_ERANGE if cap < m_bond. */
int mps_schmidt(mps_handle h, int bond, double* lam, int cap, int* m);

/* Double-double Schmidt coefficients (hi, lo); on an FP64 handle lo = 0. */
int mps_schmidt_dd(mps_handle h, int bond, double* lam_hi, double* lam_lo, int cap, int* m);

/* Amplitude <b_0 ... b_{n-1}|Psi> of Eq. (1); bits[q] in {0,1} is qubit q.
 * out = {re, im}. */
int mps_amplitude(mps_handle h, const unsigned char* bits, double out[2]);

/* Double-double amplitude: out = {re_hi, re_lo, im_hi, im_lo}. */
int mps_amplitude_dd(mps_handle h, const unsigned char* bits, double out[4]);

/* `count` amplitudes at once: bits is count x n (row per bitstring); out holds
 * 2 doubles per amplitude (FP64 handle) or 4 (dd handle: re_hi, re_lo, im_hi, im_lo). */
int mps_amplitudes(mps_handle h, int count, const unsigned char* bits, double* out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mps_amplitudes with the same arguments,
 * layout and results, bit for bit, but no device, pinned or host allocation.  Its
 * scratch (bitstrings, the site-pointer and row-length tables, the results) is a
 * fixed 4 MiB device array held by each GPU the library runs on until the process
 * ends; the bitstrings are copied straight from `bits` and the results straight
 * into `out` (pageable copies on the handle's stream, which is synchronised before
 * return).  Limit: align256(count * n) + align256(16 n) + align256(4 n) +
 * align256(count * 16) (x2 for the results of a dd handle) <= 4 MiB, else
 * MPS_ERANGE; e.g. n = 60 allows count <= 55000 on an FP64 handle.  Nothing in the
 * scratch needs to start at zero (every result is written); the array keeps the
 * last call's contents.  Calls that overlap on one GPU (handles on different
 * streams, or different threads) share the array and race: serialise them.
 * Errors as mps_amplitudes, plus MPS_EDEVICE if the array's address cannot be
 * looked up. */
int mps_amplitudes_noalloc(mps_handle h, int count, const unsigned char* bits, double* out);

/* Reduced density operator (paper, Section 3.2: RDO(list)) of `count` distinct
 * qubits q[0..count-1], 1 <= count <= 7: rho = Tr over every other qubit of
 * |Psi><Psi|, contracted exactly from the site tensors (no canonical form assumed;
 * for a normalised state Tr rho = 1).  rho is 2^count x 2^count complex, row-major,
 * interleaved (re, im): rho[r][c] = <r|rho|c> with r = sum_t i_{q[t]} 2^{count-1-t}
 * (q[0] is the most significant bit), 2 * 4^count doubles.  On a dd handle mps_rdo
 * returns hi + lo rounded to binary64.
 * Errors: MPS_EINVAL (count out of range, a qubit out of range or repeated, NULL),
 * MPS_ERANGE (the contraction needs more device memory than the workspace cap:
 * about 4^count x 16 bytes per element of a bond's m x m). */
int mps_rdo(mps_handle h, int count, const int* q, double* rho);

/* Double-double RDO: rho = rho_hi + rho_lo (same layout each; rho_lo may be NULL).
 * On an FP64 handle rho_lo receives zeros. */
int mps_rdo_dd(mps_handle h, int count, const int* q, double* rho_hi, double* rho_lo);

/* RDO_block(first, last) of the paper: the RDO of qubits first, first+1, ..., last. */
int mps_rdo_block(mps_handle h, int first, int last, double* rho);

/* Diagnostics of the last split. */
int mps_stats(mps_handle h, struct mps_update_stats* s);

/* --- state import / export (B, V) gauge ---------------------------------------- */

/* Replace the state.  dims[s] = m_s (s = 0..n-2, each <= the bond's capacity
 * min(chi_max, 2^{s+1}, 2^{n-1-s})).  B[s] points to m_{s-1} * 2 * m_s complex
 * values, row-major [alpha][i][beta], interleaved (re, im); lam[s] to m_s values.
 * B_lo / lam_lo: NULL, or the lo planes on a dd handle. */
int mps_load(mps_handle h, const int* dims, const double* const* B, const double* const* B_lo,
             const double* const* lam, const double* const* lam_lo);

/* Copy site tensor s (m_{s-1} * 2 * m_s complex) to host; lo may be NULL. */
int mps_get_site(mps_handle h, int s, double* hi, double* lo, long cap_doubles);

/* --- checkpoint and resume --------------------------------------------------------- */

/* Write the state as a self-contained byte image into buf (cap bytes): n, chi_max,
 * eps, precision, the bond dims, every bond's Schmidt values and every site tensor
 * (lo planes included on dd handles), then a 64-bit FNV-1a hash of the image.
 * *size receives the image size; with buf NULL only the size is computed.  Engine
 * options are not part of the image.  Synchronises the handle's stream.
 * Errors: MPS_EINVAL (h or size NULL), MPS_ERANGE (cap too small), MPS_EDEVICE. */
int mps_export(mps_handle h, void* buf, long cap, long* size);

/* A new handle holding the state of an image written by mps_export (of this or
 * another process), with the image's n, chi_max, eps and precision, on hip_stream
 * (NULL: a stream of its own).  Applying the same gates to it and to the exported
 * handle gives bit-identical results.  NULL on error (bad magic, version, header,
 * size or hash); the message is mps_last_error(NULL).  The caller keeps buf. */
mps_handle mps_import(const void* buf, long size, void* hip_stream);

/* --- control --------------------------------------------------------------------- */

/* Options (enum mps_option) apply to the handle's engine: for a member of a
 * batch, to the whole batch. */
int mps_set_option(mps_handle h, int key, double value);

/* Wait for all work queued on the handle's stream. */
int mps_sync(mps_handle h);

/* With MPS_OPT_KERNEL_TIMING on, accumulated device time (ms, from HIP events
 * recorded on the handle's stream around each launch) and launch count of kernel
 * class `cls` (0 theta, 1 jacobi step, 2 truncate, 3 split, 4 single-site gate,
 * 5 amplitude, 6 dd refinement, 7 reduced density operators); reset = 1 clears the
 * counters after reading.
 * cls 8 / 9 are counters (always on): *launches receives the number of
 * update-sweeps executed by the FP64 Jacobi / the dd polish (one update taking
 * one sweep counts 1), *ms receives 0.  cls 10 counts the SVD splits finalised
 * at a sweep limit (each one also made its call return MPS_ENOCONV).  cls 11
 * counts the graph replays of Jacobi sweeps (MPS_OPT_GRAPH), *ms receiving the
 * number of graphs captured. */
int mps_kernel_time(mps_handle h, int cls, double* ms, long* launches, int reset);

/* Message for the last error on h (h may be NULL: the last error of mps_create*). */
const char* mps_last_error(mps_handle h);

/* Library version string. */
const char* mps_version(void);

/* The key under which the tuning table (the per-size Jacobi step configurations
 * chosen by the package's autotuner) is looked up for the current device: its
 * architecture and the HIP runtime version, e.g. "gfx950 70226015"; "" if the
 * device cannot be queried.  The table is read from $MPS_TUNING_FILE, else from
 * tuning.txt beside the library; a handle created on a device with no matching
 * section uses the defaults of MPS_OPT_BLOCK_WIDTH, MPS_OPT_MAX_INNER_FEW and
 * MPS_OPT_QR, and setting any of those three options on a handle replaces the
 * table's choices for it. */
const char* mps_tuning_key(void);

/* --- batches of independent circuits ----------------------------------------------
 * Many states evolved by independent circuits, updated together: the library's
 * scheduler takes the gates of all circuits at once, so updates of different
 * circuits share every launch (one Jacobi step launch serves all iterating
 * updates of all circuits).  Each circuit's gates keep their order where they
 * share sites, so each state ends exactly as if its circuit ran alone on a handle
 * of the same precision, chi_max and eps. */
typedef struct mps_batch* mps_batch_handle;

/* `count` states |0...0>: circuit i has n[i] qubits, chi_max[i], eps[i]; all share
 * one precision and one HIP stream.  All state memory is one device allocation.
 * Returns NULL on error (see mps_batch_last_error(NULL)). */
mps_batch_handle mps_batch_create(int count, const int* n, const int* chi_max, const double* eps, int prec);

/* Apply `ngates` gates: gate g acts on circuit[g] at sites first[g]..first[g]+k[g]-1,
 * U (and U_lo: NULL, or the lo parts on a dd batch) packed back to back as in
 * mps_apply_gates.  Every gate is checked before any runs.  Errors as
 * mps_apply_gates; messages via mps_batch_last_error. */
int mps_batch_run(mps_batch_handle b, long ngates, const int* circuit, const int* first, const int* k,
                  const double* U, const double* U_lo);

/* The state of circuit i, for every readout call of this header (and for gates
 * applied to it alone).  The batch owns it: do not pass it to mps_destroy. */
mps_handle mps_batch_get(mps_batch_handle b, int circuit);

int mps_batch_set_option(mps_batch_handle b, int key, double value);
const char* mps_batch_last_error(mps_batch_handle b);
int mps_batch_destroy(mps_batch_handle b);

#ifdef __cplusplus
}
#endif

#endif /* MPS_H_ */
