// Internal launch interface between the C ABI / host drivers and the HIP
// kernels of libhrd.  Nothing here is exported.
#pragma once

#include "common.h"

namespace hrd {

// ----- hopping stencil (dslash.hip) ---------------------------------------
struct HopArgs {
    Geom g;
    const void *U;      // packed gauge field
    const char *src;    // source field (opposite parity); FULL: full-lattice psi
    const char *self;   // HAS_A: target-parity field for the a*psi term
    char *dst;          // output (target parity); FULL: full-lattice out
    double a, b;        // out = a * self + b * (H src)
    double *partials;   // NORM: one ||out||^2 partial per block
    int parity;         // target parity (ignored by FULL)
    size_t half_bytes;  // FULL: bytes of one parity block of a spinor
    void *r;            // RUPD: residual updated in place, r <- r - alpha * out
    const double *sc;   // RUPD: device scalars (alpha in slot S_ALPHA)
    const void *clov;   // clover epilogues: packed site matrices of the target parity's field
    int rel;            // FP64 SU(2) formats: every spinor and link block is below 2 GiB, so
                        // loads address it with 32-bit offsets (set by launch_hop)
};

// Clover epilogues of the hopping kernel (the site matrix M = m + A is read
// from HopArgs::clov, precision of the launch):
//   CLOV_SELF:  out = M self + b (H src)          (replaces a * self)
//   CLOV_INV:   out = M (b (H src))               (clov holds M^{-1})
enum CloverMode { CLOV_NONE = 0, CLOV_SELF = 1, CLOV_INV = 2 };

int hop_blocks(const Geom &g);
// Sites per workgroup of the hopping kernels of one format and precision:
// 64 for the FP64 kernels of the SU(2) formats (one-wave workgroups) and of
// CPLX10 (four lanes per site), 256 for every other kernel.  A launch that
// writes ||out||^2 partials writes one per workgroup,
// hop_partials(rep, prec, g) = ceil(Vh / sites) of them.
constexpr int hop_sites_per_block(int rep, int prec)
{
    return (prec == HRD_F64 && (!is_dense(rep) || rep == HRD_CPLX10)) ? 64 : 256;
}
int hop_partials(int rep, int prec, const Geom &g);
hipError_t launch_hop(int rep, int prec, const HopArgs &a, bool dag, bool has_a, bool norm, bool full,
                      hipStream_t st, int clov = CLOV_NONE);
// Second stage of D^+ fused with the CG residual update: out = a self + b H src
// is not stored; instead r <- r - alpha out and ||r||^2 partials are written
// (one per workgroup, hop_partials(rep, prec, g) of them).
hipError_t launch_hop_rupdate(int rep, int prec, const HopArgs &a, hipStream_t st, int clov = CLOV_NONE);
// the same for the dense SU(N > 2) formats (clover only for CPLX3 and
// SU3_ROW2), dslash_sun.hip
hipError_t launch_hop_dense(int rep, int prec, const HopArgs &a, bool dag, bool has_a, bool norm, bool full,
                            hipStream_t st, int clov);
hipError_t launch_hop_rupdate_dense(int rep, int prec, const HopArgs &a, hipStream_t st, int clov);

// ----- field preparation (pack.hip) ----------------------------------------
hipError_t launch_pack_spinor(int rep, int prec, int sites, const Geom &g, const void *nat, void *packed,
                              bool unpack, hipStream_t st);
hipError_t launch_pack_gauge(int rep, int prec, const Geom &g, const void *nat, void *packed, bool unpack,
                             hipStream_t st);
hipError_t launch_represent(int prec_out, const Geom &g, const void *Uf, void *Ua, hipStream_t st);
hipError_t launch_represent_backward(const Geom &g, const void *Uf, const void *ga, void *Gf, hipStream_t st);
hipError_t launch_convert_gauge(int rep, const Geom &g, const void *U64, void *U32, hipStream_t st);
// nparity blocks of Vh sites, ncomp complex components per site
hipError_t launch_convert_spinor(int Vh, int nparity, int ncomp, bool to_f32, const void *in, void *out,
                                 hipStream_t st);
// dense SU(N > 2) formats (pack_sun.hip): natural <-> packed, F64 -> F32/F16,
// and the representations of fundamental SU(nc) links (CPLXnc, F64) in the
// format of the representation (F64): kind 0 fund, 1 adj, 2 sym, 3 asym
hipError_t launch_pack_gauge_dense(int rep, int prec, const Geom &g, const void *nat, void *packed, bool unpack,
                                   hipStream_t st);
hipError_t launch_convert_gauge_dense(int rep, int prec_out, const Geom &g, const void *U64, void *Uout,
                                      hipStream_t st);
// chain rule of launch_represent_sun: G_rep (format of the representation,
// FP64) -> G_fund (CPLXnc, FP64)
hipError_t launch_represent_backward_sun(int nc, int kind, const Geom &g, const void *Uf, const void *Gr, void *Gf,
                                         hipStream_t st);
hipError_t launch_represent_sun(int nc, int kind, const Geom &g, const void *Uf, void *Ur, hipStream_t st);
// F64 links -> F16 links
hipError_t launch_convert_gauge_h16(int rep, const Geom &g, const void *U64, void *U16, hipStream_t st);
// spinor storage conversion between any two precisions (same precision: copy)
hipError_t launch_convert_spinor_prec(int rep, int Vh, int nparity, int prec_in, int prec_out, const void *in,
                                      void *out, hipStream_t st);

// ----- level-1 linear algebra (blas.hip) ------------------------------------
// All reductions write kRedBlocks partials; finalize_* sums them in a fixed
// order on one block.
constexpr int kRedBlocks = 1024;

// Complex-pair view of a packed field: n complex numbers, F64 or F32.
hipError_t launch_dot_partials(int prec, size_t n, const void *a, const void *b, double *partials,
                               hipStream_t st);  // 2 partials per block (re, im)
hipError_t launch_norm_partials(int prec, size_t n, const void *a, double *partials, hipStream_t st);
hipError_t launch_axpy(int prec, size_t n, double ar, double ai, const void *x, void *y, double *partials,
                       hipStream_t st);  // partials may be null
hipError_t launch_xpay(int prec, size_t n, const void *x, double ar, double ai, void *y, hipStream_t st);
// sums[0..ncol) = column sums of a [nblk][ncol] partial table
hipError_t launch_finalize(const double *partials, int nblk, int ncol, double *sums, hipStream_t st);

// ----- CG building blocks (blas.hip) -----------------------------------------
// Device scalar slots used by the CG drivers.
enum ScalarSlot {
    S_RR = 0,      // current ||r||^2
    S_PAP = 1,     // <p, A p> = ||D^ p||^2
    S_ALPHA = 2,   // rr / pAp
    S_BETA = 3,    // rr_new / rr
    S_RRNEW = 4,   // ||r_new||^2
    S_FLAG = 5,    // breakdown flag (non-zero)
    S_BB = 6,      // ||b||^2
    S_RROLD = 7,   // ||r||^2 before the last beta stage
    S_COUNT = 8
};
// Sum partials of ||D^p||^2 and set alpha = rr / pAp (flag breakdown); also
// store alpha at *hist when hist is not null.
hipError_t launch_cg_alpha(const double *partials, int nblk, double *sc, hipStream_t st, double *hist = nullptr);
// Sum partials of ||r||^2 into rr_new and set beta = rr_new / rr, rr = rr_new.
hipError_t launch_cg_beta(const double *partials, int nblk, double *sc, hipStream_t st);
// r <- r - alpha Ap (F64 or F32 fields), partials of ||r||^2 (FP64).
hipError_t launch_cg_update_r(int prec, size_t n, void *r, const void *Ap, const double *sc, double *partials,
                              hipStream_t st);
// F64 CG: x <- x + alpha p ; p <- r + beta p.
hipError_t launch_cg_update_xp64(size_t n, void *x, void *p, const void *r, const double *sc, hipStream_t st);
// p32 <- r32 + beta p32 with beta = rr / rr_old (batched CG, after a reliable update).
hipError_t launch_cg_update_p32(size_t n16, void *p32, const void *r32, const double *sc, hipStream_t st);
// Mixed CG search directions: a ring of kPRing low-precision (F32 or F16)
// fields, `stride` bytes apart, whose solution updates are deferred.  Flush
// (m > 0): x64 += alpha_s p_s for the slots s = 0 .. m-1 in order,
// alpha_s = ahist[s].  Advance (dst >= 0, after the flush when both):
// p_dst = r32 + beta p_src with beta = sc[S_BETA] (kBetaIter), rr / rr_old
// (kBetaRatio, after a reliable update) or 0 (kBetaZero, restart).
constexpr int kPRing = 8;
// Default reliable-update thresholds (delta <= 0).  The solution accumulates
// in FP64, so only the low-precision recurrence of r drifts from the true
// residual: for FP32 operator fields the drift stays far below 1e-3 of the
// residual a cycle starts from, for F16 fields it is of order 1e-3 per cycle.
constexpr double kDeltaMixed = 1e-3;
constexpr double kDeltaMixed16 = 3e-2;
enum RingBeta { kBetaIter = 0, kBetaRatio = 1, kBetaZero = 2 };
hipError_t launch_cg_ring(int prec, int Vh, int ncomp, void *x64, void *ring, size_t stride, int m, int src,
                          int dst, const void *r32, const double *sc, const double *ahist, int beta_mode,
                          hipStream_t st);
// Reliable update: r64 = b - Ax64 ; r32 = f32(r64) ; partials of ||r64||^2.
hipError_t launch_cg_residual_mixed(int Vh, int ncomp, const void *b, const void *Ax, void *r64, void *r32,
                                    double *partials, hipStream_t st);
// r = b - Ax (F64), partials of ||r||^2.
hipError_t launch_cg_residual64(size_t n, const void *b, const void *Ax, void *r, double *partials,
                                hipStream_t st);
// p32 <- r32 (copy) ; used at (re)starts.
hipError_t launch_copy(size_t bytes, const void *src, void *dst, hipStream_t st);
// dst = 0
hipError_t launch_zero(size_t bytes, void *dst, hipStream_t st);

// ----- clover term (clover.hip) ---------------------------------------------
// M = m + A (or m exp(A/m)) and M^{-1} of every site from the F64 links of
// the representation.
hipError_t launch_clover_build(int rep, bool exponential, const Geom &g, const void *U, double csw, double m, void *M,
                               void *Minv, hipStream_t st);
hipError_t launch_convert_clover(int rep, const Geom &g, const void *C64, void *C32, hipStream_t st);
// packed F64 -> complex128 [V][4N][4N], lexicographic sites
hipError_t launch_unpack_clover(int rep, const Geom &g, const void *C, void *nat, hipStream_t st);

// ----- force (force.hip) ---------------------------------------------------
hipError_t launch_force(int rep, const Geom &g, const void *X, const void *Y, void *F, double scale,
                        hipStream_t st);

}  // namespace hrd
