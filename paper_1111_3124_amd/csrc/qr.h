// Launchers of the QR preconditioning of wide thetas (M < Nt).
#pragma once
#include "common.h"

namespace mpsk {

// theta_w^H = Q R for each listed task: R^H (M x M) becomes the Jacobi matrix in
// thw (and, dd, in Rh), Q (Nt x M) is left in Qh; one 1024-thread block per task
hipError_t launch_qr(Task2* d_tasks, const Ent* d_ents, int nent, bool dd, hipStream_t st);
// after the truncation: Z[:, nu] = Q V_R[:, perm[nu]], nu < k (the kept count)
hipError_t launch_zform(Task2* d_tasks, const Ent* d_ents, int nent, int maxNt, int maxK, bool dd, hipStream_t st);

}  // namespace mpsk
