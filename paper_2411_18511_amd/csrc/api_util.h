// Host-side helpers shared by the C-ABI implementation files: error
// reporting, argument checks and the operator compositions.
#pragma once

#include <algorithm>

#include "kernels.h"

#define HRD_TRY(expr)                       \
    do {                                    \
        const hrd_status s__ = (expr);      \
        if (s__ != HRD_OK) return s__;      \
    } while (0)

namespace hrd {

hrd_status fail(hrd_status st, const char *fmt, ...);
hrd_status check_hip(hipError_t e, const char *what);
hrd_status check_lattice(const hrd_lattice *lat);
hrd_status check_rep_prec(hrd_rep rep, hrd_prec prec);      // F64 or F32
hrd_status check_rep_prec_any(hrd_rep rep, hrd_prec prec);  // F64, F32 or F16
hrd_status check_clover_format(hrd_rep rep, const char *what);  // EINVAL unless clover_capable(rep)
bool overlap(const void *a, size_t na, const void *b, size_t nb);
size_t spinor_bytes(const hrd_lattice *lat, int rep, int prec, int nparity);
size_t gauge_bytes(const hrd_lattice *lat, int rep, int prec);
int ncomp_of(int rep);
size_t clover_bytes(const hrd_lattice *lat, int rep, int prec);

// Packed clover fields of one precision: M = m + A and M^{-1}, both parities.
struct CloverRef {
    const void *M;
    const void *Minv;
};

// D^ (dag: D^+) of an even half field; tmp is an odd half field; optional
// ||out||^2 partials (hop_blocks(g) of them).
// With a clover field cl: D^ = M_ee - D_eo M_oo^{-1} D_oe (m0 unused).
hipError_t apply_dhat(int rep, int prec, const Geom &g, const void *U, const void *in, void *out, void *tmp,
                      double m0, bool dag, double *norm_partials, hipStream_t st, const CloverRef *cl = nullptr);
// r <- r - alpha (D^+ q), ||r||^2 partials (hop_blocks(g) of them); alpha is
// read from sc[S_ALPHA] on the device; tmp is an odd half field.
hipError_t apply_dhat_dag_update_r(int rep, int prec, const Geom &g, const void *U, const void *q, void *r, void *tmp,
                                   double m0, const double *sc, double *partials, hipStream_t st,
                                   const CloverRef *cl = nullptr);
// out (parity target) = D_{target,1-target} in, or its g5-conjugate.
hipError_t apply_hop_block(int rep, int prec, const Geom &g, const void *U, const void *in, void *out,
                           int target, bool dag, hipStream_t st);
// out = D in on full-lattice fields (with cl: D = M - H/2, m0 unused).
hipError_t apply_full(int rep, int prec, const Geom &g, const void *U, const void *in, void *out, double m0,
                      bool dag, hipStream_t st, const CloverRef *cl = nullptr);

// hrd_dirac_apply after its argument checks (work: the caller's HRD_EO
// workspace, checked for overlaps like any caller buffer).
hrd_status dirac_apply_checked(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, const void *psi,
                               void *out, double m0, hrd_parity parity, int dagger, void *work, void *stream);

}  // namespace hrd
