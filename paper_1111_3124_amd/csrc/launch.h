// Host-side launchers of the gate-update kernels (one per kernel family).
#pragma once
#include "common.h"

namespace mpsk {

struct AmpArgs {
  const double2* const* B;  // n device pointers (site tensors)
  const int* ld;            // n row lengths
  const int* dimx;          // n + 1 bond dims, dimx[0] = dimx[n] = 1
  int n;
  const unsigned char* bits;  // count x n
  double2* out;               // count
};

hipError_t launch_prep2(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st);
// ||theta_w||_F^2 of each listed task into *fro2 (after its theta kernels); maxMN: the
// largest M x Nt of the list
hipError_t launch_fro(Task2* d_tasks, const Ent* d_ents, int nent, long maxMN, hipStream_t st);
hipError_t launch_theta2(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st);
// phase_clock: NULL, or 5 long longs receiving wall_clock64() stamps of block (0, 0)
// (start, after Gram, after inner Jacobi, end, rotated?) for phase profiling
// defer (block width 8): V's update of each step is left to the next step's launch,
// whose grid then holds a second block a pair; launch_jacobi_vflush applies the last
// step's after a launch sequence
hipError_t launch_jacobi_step(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int bw, int step, double tol_mult,
                              int maxin, int maxin_few, int defer, hipStream_t st, long long* phase_clock = nullptr);
// V's rotations still deferred after the listed tasks' sweep (the list of that sweep)
hipError_t launch_jacobi_vflush(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st);
// the same step as two launches (partial Grams, then rotations and updates) of two
// 256-thread blocks a column-block pair; block width 8
hipError_t launch_jacobi_split(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int step, double tol_mult,
                               int maxin, int maxin_few, hipStream_t st);
// column order of each task's sweep (sorted by the previous sweep's column norms)
hipError_t launch_jacobi_order(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st);
// QR preconditioning (tasks with qr set): theta_w's columns ordered by norm, the
// blocked Householder QR in place, X = R^H into the Jacobi's W operand
hipError_t launch_qr_order(Task2* d_tasks, const Ent* d_ents, int nent, hipStream_t st);
hipError_t launch_qr_factor(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, hipStream_t st);
// after the Jacobi: the Jacobi's V (N x N) <- Q V (the left singular vectors)
hipError_t launch_qr_left(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, hipStream_t st);
// after the truncation: Z's kept columns from the normalised columns of W, rows by qperm
hipError_t launch_qr_z(Task2* d_tasks, const Ent* d_ents, int nent, int maxN, int maxK, hipStream_t st);
// chi_max and eps are read from each task
hipError_t launch_truncate(Task2* d_tasks, const Ent* d_ents, int nent, double floor_rel, hipStream_t st);
// right = false: only B_s' (the first split of a three-site gate)
hipError_t launch_split(Task2* d_tasks, const Ent* d_ents, int nent, int maxM, int maxN, int maxK, hipStream_t st,
                        bool right = true);
// wide thetas, after the truncation: the kept columns of W scaled to unit norm (Z)
hipError_t launch_znorm(Task2* d_tasks, const Ent* d_ents, int nent, int maxJM, int maxK, hipStream_t st);
hipError_t launch_gate1(Task1* d_tasks, int ntask, long maxel, hipStream_t st);
hipError_t launch_amplitude(const AmpArgs& args, int count, hipStream_t st);
// *ones[i] = 1.0 for i < n_ones; dims[i] = 1 for i < n_dims (one launch for many states)
hipError_t launch_set_product(double* const* ones, long n_ones, int* dims, long n_dims, hipStream_t st);

}  // namespace mpsk
