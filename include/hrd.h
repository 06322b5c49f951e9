/*
 * hrd.h — C ABI of libhrd, an MI355X (gfx950) library for the Wilson-Dirac
 * operator of SU(2) lattice gauge theory with fermions in the fundamental or
 * adjoint representation, its even/odd preconditioned form, conjugate-gradient
 * solvers on D^+D^ (FP64 and mixed precision), the fermion force, and batched
 * multi-right-hand-side / mixed-volume variants.
 *
 * Paper: arXiv:2411.18511, "Scaling SU(2) to 1000 GPUs using HiRep".  The
 * paper benchmarks the unimproved Wilson-Dirac operator (Sec. 2.1, Table 1),
 * uses its even/odd preconditioned version inside HMC (Sec. 2.1), runs
 * fermions in higher representations (Sec. 1) and mentions a range of
 * inverters (abstract); it writes none of them down.  The definitions below
 * are the standard ones this library implements.
 *
 * ---------------------------------------------------------------------------
 * CONVENTIONS
 *   Lattice   x = (t, x1, x2, x3), extents dims = {T, L1, L2, L3}, each even
 *             and >= 2; mu = 0 is time.  V = T L1 L2 L3, Vh = V / 2.
 *   Boundary  periodic in space, antiperiodic in time, applied as the hop sign
 *             s_mu(x) = -1 iff mu = 0 and t(x) = T - 1; the links themselves
 *             stay periodic.
 *   Gammas    chiral basis in 2x2 blocks: g0 = [[0, 1], [1, 0]],
 *             gk = [[0, -i sk], [i sk, 0]] (sk Pauli matrices);
 *             g5 = g0 g1 g2 g3 = diag(-1, -1, +1, +1).
 *   Hopping   (H psi)(x) = sum_mu [ s_mu(x) (1 - g_mu) U_mu(x) psi(x + mu)
 *                                 + s_mu(x - mu) (1 + g_mu) U_mu(x - mu)^+ psi(x - mu) ]
 *   Operator  D = m - H / 2 with m = 4 + m0 (bare mass m0).
 *   Even/odd  parity(x) = (t + x1 + x2 + x3) mod 2, even = 0.  In (even, odd)
 *             blocks D = [[m, D_eo], [D_oe, m]] with D_eo = -H_eo / 2, and the
 *             preconditioned operator on even sites is the Schur complement
 *             D^ = m - (1/m) D_eo D_oe.  D^+ = g5 D^ g5.
 *   Reps      FUND: U in SU(2), 2 colours.  ADJ: R_ab(U) = tr(s_a U s_b U^+)/2,
 *             a real orthogonal 3x3 matrix, 3 colours.
 *
 * SITE ORDER (both parities)
 *   lex(x) = ((t L1 + x1) L2 + x2) L3 + x3.  A site of parity p has index
 *   lex(x) >> 1 within the parity-p block (a bijection since L3 is even).
 *
 * PACKED LAYOUTS ("library layout"; all device memory)
 *   A field of one parity is a sequence of PLANES; a plane is an array of Vh
 *   elements, one per site, in site order, except where a field is stored in
 *   TILES (below).  Spinor components are numbered k = spin * N + colour
 *   (N = 2 FUND, FUND_SU2; 3 ADJ, ADJ_SU2; 4N components).
 *     spinor, F64 : 4N planes of complex128 (16 B): plane k = component k.
 *     spinor, F32 : 2N planes of 2 x complex64 (16 B): plane k = components
 *                   (2k, 2k+1).
 *     link FUND F64: 4 planes of complex128, entries U00, U01, U10, U11.
 *     link FUND F32: 2 planes of 2 x complex64: (U00, U01), (U10, U11).
 *   TILES (every spinor field, FUND F64 and F32 links, ADJ links, and
 *     FUND_SU2 and ADJ_SU2 F64 links; the other link layouts are planes):
 *     a block of Vh
 *     sites (one parity of a spinor, one (parity, mu) of a gauge field) is
 *     split into tiles of 64 sites (the last tile: the remaining nb sites);
 *     tile t holds plane 0 of its nb sites, then plane 1, ...; element
 *     (plane q, site s) of a block with P 16-byte planes sits at byte
 *     16 (64t P + q nb + s - 64t), t = s / 64.  An F16 spinor tile holds its
 *     N planes, then the nb FP32 site scales: the scale of site s at byte
 *     64t (16N + 4) + 16 N nb + 4 (s - 64t), and plane q at
 *     64t (16N + 4) + 16 (q nb + s - 64t).  An ADJ link tile likewise holds
 *     its 16-byte planes, then the nb last entries (entry 8: float64,
 *     float32 or binary16): with P planes and E-byte entries, plane q of
 *     site s at 64t (16P + E) + 16 (q nb + s - 64t), entry 8 at
 *     64t (16P + E) + 16 P nb + E (s - 64t).  Blocks keep their sizes.
 *     link ADJ  F64: 4 planes of 2 x float64 holding entries (0,1) (2,3) (4,5)
 *                    (6,7), then 1 plane of float64 holding entry 8; entry
 *                    e = 3 a + b of R_ab.
 *     link ADJ  F32: 2 planes of 4 x float32 (entries 0-3, 4-7), then 1 plane
 *                    of float32 (entry 8).
 *     link FUND_SU2, ADJ_SU2 F64: 2 planes of complex128, entries U00, U01 of
 *                    the fundamental link.
 *     link FUND_SU2, ADJ_SU2 F32: 1 plane of 2 x complex64: (U00, U01).
 *     spinor, F16 : N planes of 16 B, each 4 components as 8 binary16
 *                   (re, im, ...) of the component divided by the site
 *                   scale s, then the float32 s (4 B per site).  s is
 *                   the largest |re| or |im| over the site's components (after
 *                   rounding them to float32); the stored value is
 *                   binary16(x * (1/s)) in float32 arithmetic, round to
 *                   nearest even; s = 0 stores zeros.  The value read back is
 *                   binary16 * s.  4N * 4 + 4 bytes per site.
 *     link FUND F16: 1 plane of 8 binary16 (U00, U01, U10, U11 as re, im).
 *     link ADJ  F16: 1 plane of 8 binary16 (entries 0-7), then 1 plane of
 *                    binary16 (entry 8).
 *     link FUND_SU2, ADJ_SU2 F16: 1 plane of 4 binary16 (U00, U01).
 *     F16 links carry no scale (entries are bounded by 1); each entry is the
 *     binary16 of its float32 rounding.
 *     link CPLXn (n x n complex, entry e = n i + j): F64 n^2 planes of
 *                    complex128; F32 ceil(n^2/2) planes of 2 x complex64
 *                    (entries 2q, 2q+1); F16 ceil(n^2/4) planes of 4 complex
 *                    as 8 binary16 (entries 4q .. 4q+3).  Slots past the last
 *                    entry are padding (written as zero).
 *     link REAL15 (15 x 15 real, entry e = 15 i + j): F64 113 planes of 2
 *                    float64, F32 57 planes of 4 float32, F16 29 planes of 8
 *                    binary16 (padding as for CPLXn).
 *     link REAL8 (8 x 8 real, entry e = 8 i + j): F64 32 planes of 2 float64,
 *                    F32 16 planes of 4 float32, F16 8 planes of 8 binary16.
 *     link SU3_ROW2 (rows 0 and 1 of an SU(3) link, entries U00 U01 U02 U10
 *                    U11 U12): F64 6 planes of complex128, F32 3 planes of
 *                    2 x complex64, F16 1 plane of 4 complex (U00 .. U10) as
 *                    8 binary16 then 1 plane of 2 complex (U11, U12) as 4
 *                    binary16.  Natural layout: complex128 [4][V][3][3].
 *   A full-lattice spinor is [parity][planes][Vh], even block first.  A
 *   gauge field is [parity][mu][planes][Vh]: block (p, mu) holds the links
 *   U_mu(x) of the sites x of parity p.
 *
 * NATURAL LAYOUTS (device memory; used only by the pack/unpack calls)
 *   spinor : complex128 [V][4][N]          (site lex, spin, colour)
 *   gauge  : complex128 [4][V][2][2] FUND, FUND_SU2 and ADJ_SU2 (the
 *            fundamental links), float64 [4][V][3][3] ADJ, complex128
 *            [4][V][n][n] CPLXn, float64 [4][V][8][8] REAL8, float64
 *            [4][V][15][15] REAL15
 *
 * OWNERSHIP AND ERRORS
 *   Every field pointer is a device pointer owned by the caller; the library
 *   never allocates device memory: temporaries come from caller-provided
 *   workspaces whose sizes the *_bytes queries return (the one exception,
 *   hrd_dirac_apply_static, keeps its temporary in a static device array).
 *   The CG solvers read their scalars through a small pinned host buffer and
 *   two events, created on a host thread's first solve on a device and kept
 *   until the process ends.  Calls are enqueued on
 *   the given stream (a hipStream_t; NULL means the null stream) and return
 *   without synchronising unless stated.  No call aborts or throws: each
 *   returns an hrd_status, and hrd_last_error() gives a thread-local message
 *   for the last failure.  Output buffers must not overlap input buffers
 *   (HRD_EALIAS).  Stream-ordered calls report launch failures (HRD_EHIP);
 *   faults inside a kernel surface at the next synchronisation.
 * ---------------------------------------------------------------------------
 */
#ifndef HRD_H
#define HRD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRD_OK = 0,
    HRD_EINVAL = 1,      /* bad enum value, NULL pointer, non-finite scalar     */
    HRD_ESHAPE = 2,      /* lattice extent odd, < 2, or too large              */
    HRD_EALIAS = 3,      /* an output buffer overlaps an input buffer          */
    HRD_EHIP = 4,        /* a HIP runtime call or kernel launch failed         */
    HRD_ENOCONV = 5,     /* solver hit maxiter before reaching the tolerance   */
    HRD_EBREAKDOWN = 6,  /* solver breakdown: <p, A p> <= 0 or NaN residual    */
    HRD_ESIZE = 7        /* caller-provided workspace too small                */
} hrd_status;

/* Fermion representation and link storage.  HRD_FUND and HRD_ADJ store the
   links of that representation.  The _SU2 variants store only the first row
   (U00, U01) of each fundamental link: an SU(2) matrix is
   [[a, b], [-conj(b), conj(a)]], so the second row is reconstructed exactly
   in the kernels, and for HRD_ADJ_SU2 the adjoint matrix R(U) is computed
   from that row inside the kernels (the quaternion form of R).  This halves
   (FUND) or cuts by 5/9 (ADJ) the link bytes the operator reads; it assumes
   the links are exactly of SU(2) form. */
typedef enum {
    HRD_FUND = 0,
    HRD_ADJ = 1,
    HRD_FUND_SU2 = 2,
    HRD_ADJ_SU2 = 3,
    /* SU(N > 2) (Sec. 1: SU(N) with fermions in higher representations):
       links of the fermion representation stored as dense matrices.  The
       representation fixes only the colour count N_R and whether links are
       complex or real:
         HRD_CPLX3 : complex 3x3 (SU(3) fundamental, SU(3) 2-index antisymmetric)
         HRD_CPLX4 : complex 4x4 (SU(4) fundamental)
         HRD_CPLX6 : complex 6x6 (SU(3) 2-index symmetric, SU(4) 2-index
                     antisymmetric)
         HRD_REAL8 : real 8x8    (SU(3) adjoint)
         HRD_CPLX10: complex 10x10 (SU(4) 2-index symmetric)
         HRD_REAL15: real 15x15  (SU(4) adjoint)
       hrd_represent_sun builds them from fundamental SU(N) links. */
    HRD_CPLX3 = 4,
    HRD_CPLX4 = 5,
    HRD_CPLX6 = 6,
    HRD_REAL8 = 7,
    /* SU(3) fundamental links stored as their first two rows; the third row
       is conj(row0 x row1), exact for SU(3) matrices (assumed). */
    HRD_SU3_ROW2 = 8,
    HRD_CPLX10 = 9,
    HRD_REAL15 = 10
} hrd_rep;
/* Storage precision of a field.  HRD_F16 is the 16-bit storage of the mixed
   solver's inner iterations (binary16 values, FP32 arithmetic; spinors carry
   a per-site FP32 scale, see PACKED LAYOUTS).  Calls that accept HRD_F16 say
   so; the others return HRD_EINVAL for it. */
typedef enum { HRD_F64 = 0, HRD_F32 = 1, HRD_F16 = 2 } hrd_prec;

/* Which block of D a call applies (Sec. 2.1: the plain operator and the
   even/odd preconditioned version). */
typedef enum {
    HRD_FULL = 0,   /* out = D psi on all V sites (full-lattice fields)          */
    HRD_EO = 1,     /* out_e = D^ psi_e (even half fields)                       */
    HRD_HOP_EO = 2, /* out_e = D_eo psi_o  (psi: odd half, out: even half)      */
    HRD_HOP_OE = 3  /* out_o = D_oe psi_e  (psi: even half, out: odd half)      */
} hrd_parity;

/* Which sites a natural-layout spinor transfer covers. */
typedef enum { HRD_SITES_ALL = 0, HRD_SITES_EVEN = 1, HRD_SITES_ODD = 2 } hrd_sites;

typedef enum { HRD_CG_F64 = 0, HRD_CG_MIXED = 1, HRD_CG_MIXED16 = 2 } hrd_cg_mode;

typedef struct {
    int dims[4]; /* {T, L1, L2, L3} */
} hrd_lattice;

typedef struct {
    int iters;                    /* CG iterations (operator applications / 2)      */
    int reliable_updates;         /* FP64 residual recomputations (mixed mode)      */
    int restarts;                 /* true-residual checks that failed and restarted */
    double true_rel_residual;     /* ||b - A x|| / ||b||, recomputed in FP64        */
    double iterated_rel_residual; /* the recursively updated residual at exit       */
    double seconds;               /* host wall time of the solve                   */
} hrd_cg_info;

/* Thread-local description of the last failure ("" if none). */
const char *hrd_last_error(void);
/* Library version string. */
const char *hrd_version(void);
/* Hash of the sources the library was built from (16 hex digits: the first
   64 bits of SHA-256 over the file names and contents of csrc/ and this
   header, in name order), so a caller can refuse a stale build.  Static
   string, never NULL. */
const char *hrd_build_hash(void);

/* ------------------------------------------------------------------------ */
/* Sizes                                                                     */
/* ------------------------------------------------------------------------ */

/* Bytes of a packed spinor on one parity (nparity = 1) or the whole lattice
   (nparity = 2).  Returns 0 for invalid arguments. */
size_t hrd_spinor_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity);

/* Bytes of a packed gauge field (all 4 V links). */
size_t hrd_gauge_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec);

/* ------------------------------------------------------------------------ */
/* Gauge preparation — links are prepared once per gauge field, as the paper
   does for its derived fields whenever the gauge field changes (Sec. 2.2).  */
/* ------------------------------------------------------------------------ */

/* Natural -> packed gauge field.  U_nat is complex128 [4][V][2][2] for FUND
   and the _SU2 formats (which keep its first row), float64 [4][V][3][3] for
   ADJ; U receives hrd_gauge_bytes(lat, rep, prec) bytes (FP32 output is
   rounded to nearest). */
hrd_status hrd_pack_gauge(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                          const void *U_nat, void *U, void *stream);

/* Packed -> natural gauge field (also used for force fields, which share the
   gauge layout).  Output dtype as for hrd_pack_gauge, always FP64; the _SU2
   formats are returned as full fundamental matrices. */
hrd_status hrd_unpack_gauge(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                            const void *U, void *U_nat, void *stream);

/* Adjoint representation of a packed FP64 fundamental field (Sec. 1, higher
   representations): U_adj(x, mu) = R(U_fund(x, mu)), R_ab = tr(s_a U s_b U^+)/2,
   written in the packed ADJ layout of precision prec_out. */
hrd_status hrd_represent(const hrd_lattice *lat, const void *U_fund, void *U_adj,
                         hrd_prec prec_out, void *stream);

/* Representations of SU(N > 2) (Sec. 1).  kind selects the representation;
   hrd_sun_rep_format returns the link format of (nc, kind), or -1 when none
   exists:  SU(3): FUND -> HRD_CPLX3, ADJ -> HRD_REAL8, SYM -> HRD_CPLX6,
   ASYM -> HRD_CPLX3;  SU(4): FUND -> HRD_CPLX4, ADJ -> HRD_REAL15,
   SYM -> HRD_CPLX10, ASYM -> HRD_CPLX6.  (SU(3)
   fundamental links may also be packed directly as HRD_SU3_ROW2.)
   Bases: ADJ R_ab = 2 Re tr(T_a U T_b U^+) with T_a the generalised Gell-Mann
   matrices halved, ordered pairwise (j < k: symmetric then antisymmetric)
   then diagonal diag(1, .., 1, -l, 0, ..) / sqrt(2 l (l + 1)); SYM / ASYM
   the action U M U^T on symmetric / antisymmetric matrices in the
   orthonormal basis e_i e_i^T (SYM only), (e_i e_j^T +- e_j e_i^T)/sqrt(2),
   pairs (i, j) row-major.  The operator's spectrum does not depend on the
   basis. */
typedef enum { HRD_SUN_FUND = 0, HRD_SUN_ADJ = 1, HRD_SUN_SYM = 2, HRD_SUN_ASYM = 3 } hrd_sun_rep;

int hrd_sun_rep_format(int nc, int kind);

/* U_rep (packed FP64, format hrd_sun_rep_format(nc, kind)) = the
   representation of the packed FP64 fundamental SU(nc) field U_fund (format
   HRD_CPLX3 for nc = 3, HRD_CPLX4 for nc = 4).  The links are taken as given
   (no reunitarisation).  Asynchronous. */
hrd_status hrd_represent_sun(const hrd_lattice *lat, int nc, hrd_sun_rep kind, const void *U_fund,
                             void *U_rep, void *stream);

/* Chain rule of hrd_represent_sun, so that a derivative taken with respect to
   the links of a representation (hrd_dirac_force on those links) reaches the
   fundamental SU(nc) links (the HMC force of Sec. 2.1 for fermions in the
   representations of Sec. 1).  G_rep: packed FP64 field in the format of the
   representation, a derivative G = dL/dRe R + i dL/dIm R (real for the
   adjoint); U_fund: the packed FP64 fundamental field (HRD_CPLX3 or
   HRD_CPLX4) the representation was built from; G_fund (same format as
   U_fund) receives dL/dRe U + i dL/dIm U, i.e. for L = Re sum conj(G_rep)
   R(U): FUND G_rep itself, ADJ 4 sum_ab G_ab T_a U T_b, SYM and ASYM
   2 sum_kl G_kl E_k conj(U) E_l^T (bases of hrd_represent_sun).  No overlap
   of G_fund with the inputs (HRD_EALIAS); HRD_EINVAL for an (nc, kind)
   without a format.  Asynchronous. */
hrd_status hrd_represent_backward_sun(const hrd_lattice *lat, int nc, hrd_sun_rep kind,
                                      const void *U_fund, const void *G_rep, void *G_fund,
                                      void *stream);

/* Chain rule through the adjoint map: given the packed FP64 fundamental field
   U_fund and a packed FP64 ADJ field g = dL/dR (real), writes the packed FP64
   FUND field G_fund = dL/dRe U + i dL/dIm U = sum_ab g_ab s_a U s_b. */
hrd_status hrd_represent_backward(const hrd_lattice *lat, const void *U_fund,
                                  const void *g_adj, void *G_fund, void *stream);

/* Packed FP64 -> packed FP32 gauge field (round to nearest). */
hrd_status hrd_convert_gauge(const hrd_lattice *lat, hrd_rep rep, const void *U64,
                             void *U32, void *stream);

/* ------------------------------------------------------------------------ */
/* Spinor transfers                                                          */
/* ------------------------------------------------------------------------ */

/* Natural complex128 [V][4][N] -> packed.  sites = ALL writes a full-lattice
   packed field; EVEN / ODD write a one-parity packed field from the sites of
   that parity (the other sites of psi_nat are not read). */
hrd_status hrd_pack_spinor(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                           hrd_sites sites, const void *psi_nat, void *psi,
                           void *stream);

/* Packed -> natural complex128 [V][4][N].  For EVEN / ODD only the sites of
   that parity are written; the others are left untouched. */
hrd_status hrd_unpack_spinor(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                             hrd_sites sites, const void *psi, void *psi_nat,
                             void *stream);

/* Precision conversion of nparity (1 or 2) parities of packed spinor:
   to_f32 != 0: F64 -> F32 (round to nearest); else F32 -> F64 (exact). */
hrd_status hrd_convert_spinor(const hrd_lattice *lat, hrd_rep rep, int nparity,
                              int to_f32, const void *in, void *out, void *stream);

/* Spinor storage conversion between any two of HRD_F64, HRD_F32, HRD_F16
   (nparity = 1 half field, 2 full field; same precision copies).  To F16:
   each value is rounded to float32 and the site is encoded as stated under
   PACKED LAYOUTS; from F16 to F64 the stored value binary16 * s is exact,
   to F32 it is rounded once.  Asynchronous. */
hrd_status hrd_convert_spinor_prec(const hrd_lattice *lat, hrd_rep rep, int nparity,
                                   hrd_prec prec_in, hrd_prec prec_out, const void *in,
                                   void *out, void *stream);

/* Packed FP64 gauge field -> packed HRD_F32 or HRD_F16 copy (F16: each entry
   binary16 of its float32 rounding).  Asynchronous. */
hrd_status hrd_convert_gauge_prec(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec_out,
                                  const void *U64, void *U_out, void *stream);

/* ------------------------------------------------------------------------ */
/* The operator (Sec. 2.1: unimproved Wilson-Dirac operator and its even/odd
   preconditioned version).                                                  */
/* ------------------------------------------------------------------------ */

/* Workspace bytes hrd_dirac_apply needs: one odd half field for HRD_EO, 0
   otherwise. */
size_t hrd_dirac_workspace_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                                 hrd_parity parity);

/* out = X psi with X = D, D^, D_eo or D_oe as selected by `parity`; with
   dagger != 0, X is replaced by g5 X g5 (= X^+ for FULL and EO; for
   HOP_EO it is (D_oe)^+, for HOP_OE it is (D_eo)^+).  U is the packed gauge
   field of (rep, prec); psi and out are packed spinors of the sizes the
   parity mode implies; work holds hrd_dirac_workspace_bytes bytes (may be
   NULL when that is 0).  prec may be HRD_F16 (fields in F16 storage, FP32
   arithmetic, outputs re-encoded per site).  Asynchronous. */
hrd_status hrd_dirac_apply(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                           const void *U, const void *psi, void *out, double m0,
                           hrd_parity parity, int dagger, void *work, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): hrd_dirac_apply without
   a workspace argument.  HRD_EO keeps its odd temporary in a static device
   array of hrd_dirac_static_scratch_bytes() bytes (64 MiB) that each device
   the library runs on holds until the process ends; an HRD_EO call whose
   temporary (hrd_dirac_workspace_bytes) exceeds it returns HRD_ESIZE.  The
   other parity modes use no temporary.  The array is shared by every call on
   a device, so calls that overlap on one device (different streams not
   ordered by the caller) race; it holds the last call's temporary, which
   every call rewrites before reading.  Never allocates or frees memory; the
   first call on a device looks up the array's device address.  Results equal
   hrd_dirac_apply's bit for bit (same kernels).  Asynchronous. */
size_t hrd_dirac_static_scratch_bytes(void);
hrd_status hrd_dirac_apply_static(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                                  const void *U, const void *psi, void *out, double m0,
                                  hrd_parity parity, int dagger, void *stream);

/* ------------------------------------------------------------------------ */
/* Level-1 linear algebra on packed spinors (the building blocks of the
   inverters, abstract).  n_parity = 1 or 2 selects half or full fields.
   Reductions accumulate in FP64 with a fixed-order two-stage tree, so results
   are bitwise reproducible; they synchronise the stream and return on the
   host.  `work` holds hrd_blas_workspace_bytes() bytes.                     */
/* ------------------------------------------------------------------------ */

size_t hrd_blas_workspace_bytes(void);

/* result[0] + i result[1] = <a, b> = sum conj(a) b. */
hrd_status hrd_blas_dot(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity,
                        const void *a, const void *b, double *result, void *work,
                        void *stream);

/* *result = ||a||^2. */
hrd_status hrd_blas_norm2(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity,
                          const void *a, double *result, void *work, void *stream);

/* y <- y + (a_re + i a_im) x; if result != NULL also returns ||y||^2 (fused,
   synchronising); otherwise asynchronous. */
hrd_status hrd_blas_axpy(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity,
                         double a_re, double a_im, const void *x, void *y,
                         double *result, void *work, void *stream);

/* y <- x + (a_re + i a_im) y.  Asynchronous. */
hrd_status hrd_blas_xpay(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity,
                         const void *x, double a_re, double a_im, void *y, void *stream);

/* ------------------------------------------------------------------------ */
/* Conjugate gradients on A = D^+ D^ over even sites (abstract: inverters;
   Sec. 2.1: the even/odd operator used in the HMC).                         */
/* ------------------------------------------------------------------------ */

/* Workspace bytes for hrd_cg_solve in the given mode. */
size_t hrd_cg_workspace_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode);

/* Solves A x = b.  b and x are packed FP64 even half fields; x holds the
   initial guess on entry (zero it for x0 = 0) and the solution on exit.
   U64 is the packed FP64 gauge field; U32 its packed reduced-precision copy:
   FP32 for HRD_CG_MIXED, F16 for HRD_CG_MIXED16 (hrd_convert_gauge_prec),
   ignored for HRD_CG_F64.  Stops when the true relative residual
   ||b - A x|| / ||b||, recomputed in FP64, is <= tol.
     HRD_CG_F64     : every vector and reduction in FP64.
     HRD_CG_MIXED   : iterations in FP32 (operator, r, p, A p), FP64 solution
                      accumulation and reductions, and a reliable update (FP64
                      recomputation of the residual) whenever the iterated
                      residual drops below delta times its largest value since
                      the last update (delta <= 0 selects 1e-3).  A reliable
                      update that finds the true residual above twice the
                      iterated one restarts the search direction from r
                      (counted in info->restarts) and multiplies delta by 10
                      (at most 0.5) for the rest of the solve.
     HRD_CG_MIXED16 : as HRD_CG_MIXED with the operator's fields (p, the odd
                      intermediate, D^ p) and the links in F16 storage (FP32
                      arithmetic); the iterated residual stays FP32; delta <= 0
                      selects 3e-2.
   The workspace of the mixed modes holds 8 low-precision search directions
   whose solution updates are applied to x together (the same FP64 sums in
   the same order as one update per iteration).
   maxiter bounds the iterations.  info (may be NULL) is filled in every case.
   Synchronises the stream.  Returns HRD_ENOCONV if the tolerance is not
   reached, HRD_EBREAKDOWN on <p, A p> <= 0 or a non-finite residual. */
hrd_status hrd_cg_solve(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode,
                        const void *U64, const void *U32, const void *b, void *x,
                        double m0, double tol, int maxiter, double delta,
                        void *work, size_t work_bytes, hrd_cg_info *info, void *stream);

/* ------------------------------------------------------------------------ */
/* Clover (Sheikholeslami-Wohlert) improvement: Sec. 2.2 adds to the Wilson
   operator a term diagonal in the sites and precomputes the fields it needs
   once per gauge field.  The paper gives no formula; the standard one is
     A(x) = c_sw (i/4) sum_{mu != nu} sigma_{mu nu} (x) F_{mu nu}(x),
     sigma_{mu nu} = (i/2) [g_mu, g_nu],  F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+)/8,
   Q_{mu nu}(x) the sum of the four same-oriented plaquettes of the (mu, nu)
   plane at x, in the links of the fermion representation, and
     D_sw = M - H/2 with the site matrix M(x) = m + A(x),
     D^_sw = M_ee - D_eo M_oo^{-1} D_oe on even sites,  D^_sw^+ = g5 D^_sw g5.
   M is Hermitian and commutes with g5: two Hermitian 2N x 2N blocks per site
   (spins 0,1 and spins 2,3; row (spin mod 2) N + colour).
   Formats: the four SU(2) formats (N = 2 or 3) and the SU(3) fundamental in
   HRD_CPLX3 or HRD_SU3_ROW2 (N = 3, the clover-improved QCD operator); every
   clover entry point returns HRD_EINVAL for the other dense formats.
   PACKED CLOVER FIELD (M or M^{-1}, one precision): per site and block the
   2N real diagonal entries, then the N(2N-1) complex entries below the
   diagonal in row order ((i, j), i > j, at i(i-1)/2 + j) as (re, im): 4N^2
   reals per block, 8N^2 per site, upper block first.  The field is
   [parity][planes][Vh] with planes of 16-byte elements holding consecutive
   reals (2 float64 or 4 float32).  NATURAL clover layout (hrd_unpack_clover):
   complex128 [V][4N][4N], row and column index spin * N + colour.         */
/* ------------------------------------------------------------------------ */

/* Bytes of one packed clover field (M or M^{-1}) of the given precision;
   0 for an invalid lattice, precision or a format without clover support. */
size_t hrd_clover_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec);

/* Which site matrix hrd_clover_build forms (m = 4 + m0):
     HRD_CLOVER_SW  : M = m + A (Sheikholeslami-Wohlert), M^{-1} by
                      Gauss-Jordan elimination with partial pivoting;
     HRD_CLOVER_EXP : M = m exp(A/m) (exponentiated clover, also named in
                      Sec. 2.2), M^{-1} = (1/m) exp(-A/m); each exponential by
                      scaling and squaring of a degree-16 Taylor polynomial.
   Both agree to first order in c_sw; every operator and solver below takes
   either. */
typedef enum { HRD_CLOVER_SW = 0, HRD_CLOVER_EXP = 1 } hrd_clover_kind;

/* Builds M and M^{-1} of the given kind in FP64 from the packed FP64 gauge
   field U64 of rep.  M64 and Minv64 receive hrd_clover_bytes(F64) bytes each.
   For HRD_CLOVER_SW a singular block yields non-finite entries (no error is
   raised: M is not inspected on the host).  Asynchronous. */
hrd_status hrd_clover_build(const hrd_lattice *lat, hrd_rep rep, hrd_clover_kind kind,
                            const void *U64, double csw, double m0, void *M64,
                            void *Minv64, void *stream);

/* (see also hrd_convert_spinor_prec / hrd_convert_gauge_prec for F16) */
/* FP64 -> FP32 copy of a packed clover field (for the mixed-precision CG
   and FP32 operators).  Asynchronous. */
hrd_status hrd_convert_clover(const hrd_lattice *lat, hrd_rep rep, const void *C64,
                              void *C32, void *stream);

/* Packed FP64 clover field -> natural layout (complex128 [V][4N][4N], both
   blocks and the zero off-diagonal chirality blocks written out).
   Asynchronous. */
hrd_status hrd_unpack_clover(const hrd_lattice *lat, hrd_rep rep, const void *C64,
                             void *C_nat, void *stream);

/* out = D_sw psi (HRD_FULL, full-lattice fields) or out_e = D^_sw psi_e
   (HRD_EO, even half fields; needs Minv and a workspace of
   hrd_dirac_workspace_bytes(HRD_EO) bytes); dagger != 0 applies the adjoint.
   U, M, Minv, psi and out share the precision prec, except for HRD_F16
   (F16 U, psi and out) where M and Minv are FP32.  The off-diagonal blocks
   D_eo, D_oe carry no clover term: apply them with hrd_dirac_apply
   (HRD_HOP_EO, HRD_HOP_OE gives HRD_EINVAL here).  The mass is the one built
   into M.  Asynchronous. */
hrd_status hrd_dirac_apply_clover(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                                  const void *U, const void *M, const void *Minv,
                                  const void *psi, void *out, hrd_parity parity,
                                  int dagger, void *work, void *stream);

/* CG on A = D^_sw^+ D^_sw, as hrd_cg_solve (same workspace size, same modes,
   tolerance, reliable updates, info and errors), with the FP64 clover fields
   M64, Minv64 and, for HRD_CG_MIXED and HRD_CG_MIXED16, their FP32 copies
   M32, Minv32 (ignored for HRD_CG_F64). */
hrd_status hrd_cg_solve_clover(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode,
                               const void *U64, const void *U32, const void *M64,
                               const void *Minv64, const void *M32, const void *Minv32,
                               const void *b, void *x, double tol, int maxiter, double delta,
                               void *work, size_t work_bytes, hrd_cg_info *info, void *stream);

/* ------------------------------------------------------------------------ */
/* Fermion force for the HMC (Sec. 2.1 mentions the HMC the even/odd operator
   serves).                                                                  */
/* ------------------------------------------------------------------------ */

/* F = scale * dL/dU for L = Re<X, D[U] Y>, in the convention
   dL/dU = dL/dRe U + i dL/dIm U per link entry:
     G_mu(x) = -1/2 s_mu(x) sum_spin [ X(x) (x) ((1 - g_mu) Y(x+mu))^*
                                     + ((1 + g_mu) Y(x)) (x) X(x+mu)^* ],
   (a (x) b^*)_ij = a_i conj(b_j).  X and Y are packed full-lattice FP64
   spinors; F is a packed FP64 gauge-layout field of the uncompressed
   representation (FUND for FUND and FUND_SU2, ADJ for ADJ and ADJ_SU2, the
   format itself for CPLXn and REAL8, CPLX3 for SU3_ROW2), because a
   derivative is a general matrix.  For ADJ and REAL8 the links are real and
   F = scale * Re G.  D is linear in U, so G does not depend on U;
   U is accepted so the call mirrors the operator's arguments and may be NULL.
   Asynchronous. */
hrd_status hrd_dirac_force(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec,
                           const void *U, const void *X, const void *Y, void *F,
                           double scale, void *stream);

/* Workspace bytes for hrd_action_force (two full-lattice FP64 fields). */
size_t hrd_action_force_workspace_bytes(const hrd_lattice *lat, hrd_rep rep);

/* Force of the fermion action S = phi^+ (D^+ D^)^{-1} phi given the solution
   xi = (D^+ D^)^{-1} phi (packed FP64 even half field):
     F = scale * (2/m) G[X, Y],  eta = D^ xi,  Y = (xi, D_oe xi),
     X = (eta, (D_eo)^+ eta),  m = 4 + m0,
   which is scale * dS/dU.  U is the packed FP64 gauge field of rep; F has the
   uncompressed layout as for hrd_dirac_force.  Asynchronous. */
hrd_status hrd_action_force(const hrd_lattice *lat, hrd_rep rep, const void *U,
                            const void *xi, void *F, double m0, double scale,
                            void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched multi-RHS / mixed-volume execution.  The paper advises local
   volumes of at least 16^4 for SU(2) (Sec. 3); many small problems and many
   right-hand sides are gathered into single persistent launches that read
   each link once per site for all right-hand sides of a problem.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    hrd_lattice lat;
    hrd_rep rep;
    int nrhs;          /* right-hand sides on this lattice (1..64)               */
    double m0;
    const void *U32;   /* packed FP32 gauge field                                */
    const void *U64;   /* packed FP64 gauge field (batched CG only; else NULL)   */
    const void *src;   /* nrhs consecutive packed half fields (see the calls)    */
    void *dst;         /* nrhs consecutive packed half fields                    */
} hrd_problem;

/* Launch shape of the batched kernels: sites per tile (64, 128 or 256; one
   thread per site, so also the threads per workgroup), right-hand sides
   processed per tile (1..64), workgroups per CU of the persistent grid
   (1..16), and the x1-slab width of the traversal (rounded down to a divisor
   of each problem's L1; larger than L1 means lexicographic order).  Zero
   fields select the defaults (128 sites, 4 right-hand sides, 4 workgroups per
   CU, automatic slab); other values outside these ranges give HRD_EINVAL.
   block_threads is ignored (always sites_per_tile).  hrd_autotune_batched
   tries sites {64, 128, 256} x right-hand sides {1, 2, 4, 6, 12} x
   workgroups per CU {2, 4, 8} x slabs {automatic, 1, 2, 4, 8, L1}. */
typedef struct {
    int sites_per_tile;
    int rhs_per_tile;
    int block_threads;
    int blocks_per_cu;
    int slab_width;
} hrd_tune;

/* Workspace bytes for hrd_dirac_apply_batched with parity (HRD_EO needs one
   odd FP32 temporary per right-hand side, plus the tile table). */
size_t hrd_batched_workspace_bytes(const hrd_problem *probs, int nprob, hrd_parity parity);

/* For every problem and right-hand side k: dst_k = X src_k with X as in
   hrd_dirac_apply (parity HRD_EO, HRD_HOP_EO or HRD_HOP_OE; FP32 packed half
   fields), with one persistent launch per hopping stage covering all
   problems.  Formats: the SU(2) formats (HRD_FUND, HRD_ADJ, HRD_FUND_SU2,
   HRD_ADJ_SU2) in any mix, each site's 8 links held in registers across the
   right-hand sides of a tile; or problems that all share one dense SU(N > 2)
   format, whose links are streamed by row for every right-hand side (from
   L2 after the first); any other mix is HRD_EINVAL.  tune may be NULL
   (defaults).  Asynchronous. */
hrd_status hrd_dirac_apply_batched(const hrd_problem *probs, int nprob, hrd_parity parity,
                                   int dagger, const hrd_tune *tune, void *work,
                                   size_t work_bytes, void *stream);

/* Workspace bytes for hrd_cg_solve_batched. */
size_t hrd_cg_batched_workspace_bytes(const hrd_problem *probs, int nprob);

/* Independent mixed-precision reliable-update CG solves of A x_k = b_k for
   every problem and right-hand side: src holds the FP64 packed even half
   fields b_k, dst the FP64 x_k (initial guess on entry).  The FP32 operator
   stages run batched (one launch per stage for all problems), reductions and
   scalars are per right-hand side in FP64, converged right-hand sides are
   masked out.  delta and the restart on drift as for HRD_CG_MIXED (per
   right-hand side).  infos has one entry per right-hand side, in problem
   order.
   Synchronises.  Returns HRD_ENOCONV if any system misses tol. */
hrd_status hrd_cg_solve_batched(const hrd_problem *probs, int nprob, double tol, int maxiter,
                                double delta, const hrd_tune *tune, void *work,
                                size_t work_bytes, hrd_cg_info *infos, void *stream);

/* Times candidate launch shapes of the batched hopping kernel on these
   problems (work as for hrd_dirac_apply_batched with HRD_EO; src/dst are
   overwritten) and writes the fastest to *best (median of 5 timed launches
   per candidate over tile sizes, group sizes, grid sizes and slab widths;
   ties go to the earlier, smaller candidate).  If cache_path is not NULL the
   result is looked up in / appended to that JSON-lines file, keyed by the
   GPU architecture and the problem list.  Synchronises. */
hrd_status hrd_autotune_batched(const hrd_problem *probs, int nprob, void *work,
                                size_t work_bytes, const char *cache_path, hrd_tune *best,
                                void *stream);

/* ------------------------------------------------------------------------ */
/* Bandwidth ceiling.  The operator is memory-bound (Sec. 2.1 and Table 1
   state its performance as a fraction of the device's peak bandwidth); this
   call streams a chosen read/write mix with the operator kernels' access
   instructions (16-byte non-temporal loads and stores, the same block order)
   so that the rate the device actually reaches for that mix can be measured
   beside the kernels.                                                       */
/* ------------------------------------------------------------------------ */

/* dst (write_bytes, a positive multiple of 16) receives, per 16-byte element,
   the sum (as two float64) of k = read_bytes / write_bytes source elements
   (1 <= k <= 64, read_bytes an exact multiple of write_bytes).  tiled = 0:
   the source is k consecutive streams of write_bytes each (one array per
   plane); tiled = 1: 64-element tiles, each wave reading one contiguous
   stretch of 64 k elements (write_bytes a multiple of 1024).  src and dst
   are caller-owned device buffers that must not overlap (HRD_EALIAS);
   HRD_EINVAL for sizes outside these rules.  Asynchronous. */
hrd_status hrd_stream_probe(const void *src, size_t read_bytes, void *dst, size_t write_bytes,
                            int tiled, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HRD_H */
