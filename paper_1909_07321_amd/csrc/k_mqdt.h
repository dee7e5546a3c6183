// k_mqdt.h -- launches of the quantum-defect elimination in S form (k_mqdt.hip).
#ifndef K_MQDT_H
#define K_MQDT_H
#include "rm_internal.h"

namespace rm {

// Largest number of closed members the S-form elimination inverts in LDS;
// energies with more take the route through the recovered unphysical K.
constexpr int MQDT_SMAX = 48;

// k_mqdt_setup with the lists of the S form: clist / olist the member
// positions of the closed / open members in ascending order, cch the closed
// members' channels ([e][ldo] each).
void launch_mqdt_setup_lists(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                             double thr_guard, int *syspos, int *spos, double *tanv, int *dims, int *nsys, int *status,
                             int *clist, int *olist, int *cch);
// W = (e^{-2 pi i nu} - S_cc)^-1, Z = W S_co, then (S + 1)/2 with
// S = S_oo + S_oc Z over the planes of aug that k_omega reads.  Wr, Wi:
// [ne][SMAX][SMAX]; Zr, Zi: [ne][nmax][SMAX].
void launch_mqdt_sform(hipStream_t s, const Lay &L, const DevPW *tab, const int *pwi, const double *E,
                       const int *nsys, const int *nopen, const int *clist, const int *olist, const int *cch,
                       const double *Xc, const double *Yc, const int *cidx, const double *cw, const int *status,
                       double *Wr, double *Wi, double *Zr, double *Zi, double *aug);

}  // namespace rm
#endif
