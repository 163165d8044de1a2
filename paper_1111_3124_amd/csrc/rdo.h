// Launchers of the reduced-density-operator contraction (rdo.hip).
#pragma once
#include "common.h"

namespace mpsk {

// One contraction step.  Left environment (site s with bond dims ml | mr):
// E (D blocks of ml x ml) -> F (D x 2 blocks of ml x mr) -> En (4 D or D blocks of
// mr x mr); l = listed qubits opened before this site.  Right environment: E = R
// (mr x mr), F = G (2 x ml x mr), En = R' (ml x ml).  Final: E (D x m x m), F = R
// (m x m), En = rho (D values), with mr = m.  dd: the *lo planes (else NULL).
struct RdoStep {
  const double2* B;
  const double2* Blo;
  int ld, ml, mr, l;
  const double2* E;
  const double2* Elo;
  double2* F;
  double2* Flo;
  double2* En;
  double2* Enlo;
};

hipError_t launch_rdo_left(const RdoStep& p, int D, bool open, bool dd, hipStream_t st);
hipError_t launch_rdo_right(const RdoStep& p, bool dd, hipStream_t st);
hipError_t launch_rdo_final(const RdoStep& p, int D, bool dd, hipStream_t st);

}  // namespace mpsk
