// C ABI of libhrd: argument validation, operator composition (D, D^, hop
// blocks, daggers), level-1 linear algebra, the FP64 and mixed-precision CG
// drivers and the fermion-force assembly.  Every computation runs in the HIP
// kernels of this library; this file only validates, composes and launches.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "api_util.h"
#include "clover.h"
#include "kernels.h"

namespace hrd {

thread_local std::string g_last_error;

hrd_status fail(hrd_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

hrd_status check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(HRD_EHIP, "%s: %s", what, hipGetErrorString(e));
    return HRD_OK;
}

hrd_status check_lattice(const hrd_lattice *lat)
{
    if (!lat) return fail(HRD_EINVAL, "lattice is NULL");
    long long V = 1;
    for (int i = 0; i < 4; i++) {
        const int L = lat->dims[i];
        if (L < 2 || (L & 1)) return fail(HRD_ESHAPE, "extent dims[%d] = %d must be even and >= 2", i, L);
        V *= L;
    }
    if (V > (1LL << 30)) return fail(HRD_ESHAPE, "volume %lld exceeds 2^30 sites", V);
    return HRD_OK;
}

hrd_status check_clover_format(hrd_rep rep, const char *what)
{
    if (!clover_capable(rep))
        return fail(HRD_EINVAL, "%s supports the SU(2) formats and SU(3) fundamental links only (rep %d)", what,
                    (int)rep);
    return HRD_OK;
}

hrd_status check_rep_prec_any(hrd_rep rep, hrd_prec prec)
{
    if (prec == HRD_F16) return check_rep_prec(rep, HRD_F64);
    return check_rep_prec(rep, prec);
}

hrd_status check_rep_prec(hrd_rep rep, hrd_prec prec)
{
    if (rep < HRD_FUND || rep > HRD_REAL15) return fail(HRD_EINVAL, "invalid representation %d", (int)rep);
    if (prec != HRD_F64 && prec != HRD_F32) return fail(HRD_EINVAL, "invalid precision %d", (int)prec);
    return HRD_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b || !na || !nb) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

size_t spinor_bytes(const hrd_lattice *lat, int rep, int prec, int nparity)
{
    const long long V = (long long)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    return (size_t)(V / 2) * spinor_site_bytes(rep, prec) * nparity;
}

size_t gauge_bytes(const hrd_lattice *lat, int rep, int prec)
{
    const long long V = (long long)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    return (size_t)V * 4 * link_bytes(rep, prec);
}

int ncomp_of(int rep) { return 4 * ncolour(rep); }

size_t clover_bytes(const hrd_lattice *lat, int rep, int prec)
{
    const long long V = (long long)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    return (size_t)V * clover_site_reals(ncolour(rep)) * (prec == HRD_F64 ? 8 : 4);
}

// D^ in (even half) -> out (even half), tmp: odd half of the same precision.
hipError_t apply_dhat(int rep, int prec, const Geom &g, const void *U, const void *in, void *out, void *tmp,
                      double m0, bool dag, double *norm_partials, hipStream_t st, const CloverRef *cl)
{
    const double m = 4.0 + m0;
    HopArgs a{};
    a.g = g;
    a.U = U;
    a.src = (const char *)in;
    a.self = nullptr;
    a.dst = (char *)tmp;
    a.a = 0.0;
    a.b = -0.5;
    a.parity = 1;
    // tmp = D_oe in, or M_oo^{-1} D_oe in
    if (cl) a.clov = cl->Minv;
    hipError_t e = launch_hop(rep, prec, a, dag, false, false, false, st, cl ? CLOV_INV : CLOV_NONE);
    if (e != hipSuccess) return e;
    // out = m in - (1/m) D_eo tmp, or M_ee in - D_eo tmp
    a.src = (const char *)tmp;
    a.self = (const char *)in;
    a.dst = (char *)out;
    a.a = m;
    a.b = cl ? 0.5 : 0.5 / m;
    a.parity = 0;
    a.partials = norm_partials;
    if (cl) a.clov = cl->M;
    return launch_hop(rep, prec, a, dag, true, norm_partials != nullptr, false, st, cl ? CLOV_SELF : CLOV_NONE);
}

hipError_t apply_dhat_dag_update_r(int rep, int prec, const Geom &g, const void *U, const void *q, void *r, void *tmp,
                                   double m0, const double *sc, double *partials, hipStream_t st, const CloverRef *cl)
{
    const double m = 4.0 + m0;
    HopArgs a{};
    a.g = g;
    a.U = U;
    a.src = (const char *)q;
    a.dst = (char *)tmp;
    a.a = 0.0;
    a.b = -0.5;
    a.parity = 1;
    if (cl) a.clov = cl->Minv;
    hipError_t e = launch_hop(rep, prec, a, true, false, false, false, st, cl ? CLOV_INV : CLOV_NONE);
    if (e != hipSuccess) return e;
    a.src = (const char *)tmp;
    a.self = (const char *)q;
    a.dst = nullptr;
    a.a = m;
    a.b = cl ? 0.5 : 0.5 / m;
    a.parity = 0;
    a.partials = partials;
    a.r = r;
    a.sc = sc;
    if (cl) a.clov = cl->M;
    return launch_hop_rupdate(rep, prec, a, st, cl ? CLOV_SELF : CLOV_NONE);
}

hipError_t apply_hop_block(int rep, int prec, const Geom &g, const void *U, const void *in, void *out,
                           int target, bool dag, hipStream_t st)
{
    HopArgs a{};
    a.g = g;
    a.U = U;
    a.src = (const char *)in;
    a.dst = (char *)out;
    a.a = 0.0;
    a.b = -0.5;
    a.parity = target;
    return launch_hop(rep, prec, a, dag, false, false, false, st);
}

hipError_t apply_full(int rep, int prec, const Geom &g, const void *U, const void *in, void *out, double m0,
                      bool dag, hipStream_t st, const CloverRef *cl)
{
    HopArgs a{};
    a.g = make_geom(g.L, choose_slab_full(g.L, prec));
    a.U = U;
    a.src = (const char *)in;
    a.dst = (char *)out;
    a.a = 4.0 + m0;
    a.b = -0.5;
    a.half_bytes = (size_t)g.Vh * spinor_site_bytes(rep, prec);
    if (cl) a.clov = cl->M;
    return launch_hop(rep, prec, a, dag, true, false, true, st, cl ? CLOV_SELF : CLOV_NONE);
}

}  // namespace hrd

using namespace hrd;

namespace {

// Workspace carving: 256-byte aligned sub-buffers.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    void *take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
    size_t used() const { return (off + 255) & ~(size_t)255; }
};

hrd_status read_scalars(const double *sc_dev, double *host, hipStream_t st)
{
    hrd_status s = check_hip(hipMemcpyAsync(host, sc_dev, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st),
                             "hipMemcpyAsync(scalars)");
    if (s != HRD_OK) return s;
    return check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
}

// Two pinned host copies of the CG scalars, each with an event, so that the
// host reads iteration k's scalars while the stream already runs the first
// stage of iteration k + 1.  The pinned buffer and the events are created on a
// host thread's first solve on a device and kept for the life of the process
// (one set per host thread and device), so a solve allocates nothing and
// never pays hipHostFree's implicit synchronisation.
struct PinnedScalars {
    double *h = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
};
constexpr int kMaxScalarDevices = 64;

struct ScalarPipe {
    hipStream_t st;
    double *h = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    explicit ScalarPipe(hipStream_t s) : st(s) {}
    ScalarPipe(const ScalarPipe &) = delete;
    ScalarPipe &operator=(const ScalarPipe &) = delete;
    hrd_status init()
    {
        static thread_local PinnedScalars pool[kMaxScalarDevices];
        int dev = -1;
        HRD_TRY(check_hip(hipGetDevice(&dev), "hipGetDevice"));
        if (dev < 0 || dev >= kMaxScalarDevices) return fail(HRD_EINVAL, "device ordinal %d out of range", dev);
        PinnedScalars &ps = pool[dev];
        if (!ps.ev[1]) {
            hipError_t e = hipSuccess;
            if (!ps.h) e = hipHostMalloc((void **)&ps.h, sizeof(double) * 2 * S_COUNT, hipHostMallocDefault);
            if (e == hipSuccess && !ps.ev[0]) e = hipEventCreateWithFlags(&ps.ev[0], hipEventDisableTiming);
            if (e == hipSuccess && !ps.ev[1]) e = hipEventCreateWithFlags(&ps.ev[1], hipEventDisableTiming);
            HRD_TRY(check_hip(e, "pinned CG scalars"));
        }
        h = ps.h;
        ev[0] = ps.ev[0];
        ev[1] = ps.ev[1];
        return HRD_OK;
    }
    hrd_status post(const double *sc_dev, int slot)
    {
        hrd_status s = check_hip(hipMemcpyAsync(h + slot * S_COUNT, sc_dev, sizeof(double) * S_COUNT,
                                                hipMemcpyDeviceToHost, st),
                                 "hipMemcpyAsync(scalars)");
        if (s != HRD_OK) return s;
        return check_hip(hipEventRecord(ev[slot], st), "hipEventRecord");
    }
    hrd_status wait(int slot, double *out)
    {
        HRD_TRY(check_hip(hipEventSynchronize(ev[slot]), "hipEventSynchronize"));
        std::memcpy(out, h + slot * S_COUNT, sizeof(double) * S_COUNT);
        return HRD_OK;
    }
    ~ScalarPipe()
    {
        // the next solve on this thread reuses h: no copy into it may still be in flight
        if (h) (void)hipStreamSynchronize(st);
    }
};

struct CgBuffers {
    // FP64 (every mode)
    void *r64, *p64, *q64, *Ap64, *t64;
    // mixed modes: r32 is FP32; p, q, t are FP32 (MIXED) or F16 (MIXED16);
    // plo is the ring of kPRing search directions, pstride bytes apart, and
    // ahist holds the alpha of each slot until its update is folded into x
    void *r32, *plo, *qlo, *tlo;
    size_t pstride;
    double *ahist;
    double *partials, *sc;
};

size_t carve_cg(const hrd_lattice *lat, int rep, int mode, void *work, CgBuffers *b)
{
    Carver c(work);
    const size_t h64 = spinor_bytes(lat, rep, HRD_F64, 1);
    const size_t h32 = spinor_bytes(lat, rep, HRD_F32, 1);
    const Geom g = make_geom(lat->dims);
    const int nparts = std::max(hop_partials(rep, HRD_F64, g), kRedBlocks) * 2;
    CgBuffers t{};
    t.r64 = c.take(h64);
    t.q64 = c.take(h64);
    t.Ap64 = c.take(h64);
    t.t64 = c.take(h64);
    if (mode == HRD_CG_F64) {
        t.p64 = c.take(h64);
    } else {
        const size_t hlo = mode == HRD_CG_MIXED16 ? spinor_bytes(lat, rep, HRD_F16, 1) : h32;
        t.r32 = c.take(h32);
        t.pstride = (hlo + 255) & ~(size_t)255;
        t.plo = c.take(t.pstride * kPRing);
        t.ahist = (double *)c.take(sizeof(double) * kPRing);
        t.qlo = c.take(hlo);
        t.tlo = c.take(hlo);
    }
    t.partials = (double *)c.take(sizeof(double) * nparts);
    t.sc = (double *)c.take(sizeof(double) * S_COUNT);
    if (b) *b = t;
    return c.used();
}

}  // namespace

extern "C" {

const char *hrd_last_error(void) { return g_last_error.c_str(); }

#ifndef HRD_SOURCE_HASH
#error "HRD_SOURCE_HASH must be defined by the build (hash of the library sources)"
#endif

const char *hrd_version(void) { return "hrd 0.2 (gfx950, sources " HRD_SOURCE_HASH ")"; }

const char *hrd_build_hash(void) { return HRD_SOURCE_HASH; }

size_t hrd_spinor_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec_any(rep, prec) != HRD_OK || (nparity != 1 && nparity != 2))
        return 0;
    return spinor_bytes(lat, rep, prec, nparity);
}

size_t hrd_gauge_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec_any(rep, prec) != HRD_OK) return 0;
    return gauge_bytes(lat, rep, prec);
}

hrd_status hrd_pack_gauge(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U_nat, void *U, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (!U_nat || !U) return fail(HRD_EINVAL, "NULL field pointer");
    const long long V = (long long)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    const size_t nat_bytes = (size_t)V * 4 * (rep == HRD_ADJ ? 9 * 8 : 4 * 16);
    if (overlap(U_nat, nat_bytes, U, gauge_bytes(lat, rep, prec))) return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_pack_gauge(rep, prec, g, U_nat, U, false, (hipStream_t)stream), "pack_gauge launch");
}

hrd_status hrd_unpack_gauge(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, void *U_nat, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (!U_nat || !U) return fail(HRD_EINVAL, "NULL field pointer");
    const long long V = (long long)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
    const size_t nat_bytes = (size_t)V * 4 * (rep == HRD_ADJ ? 9 * 8 : 4 * 16);
    if (overlap(U_nat, nat_bytes, U, gauge_bytes(lat, rep, prec))) return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_pack_gauge(rep, prec, g, U_nat, const_cast<void *>(U), true, (hipStream_t)stream),
                     "unpack_gauge launch");
}

hrd_status hrd_represent(const hrd_lattice *lat, const void *U_fund, void *U_adj, hrd_prec prec_out, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(HRD_ADJ, prec_out));
    if (!U_fund || !U_adj) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(U_fund, gauge_bytes(lat, HRD_FUND, HRD_F64), U_adj, gauge_bytes(lat, HRD_ADJ, prec_out)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_represent(prec_out, g, U_fund, U_adj, (hipStream_t)stream), "represent launch");
}

int hrd_sun_rep_format(int nc, int kind)
{
    if (nc == 3) {
        switch (kind) {
            case HRD_SUN_FUND: return HRD_CPLX3;
            case HRD_SUN_ADJ: return HRD_REAL8;
            case HRD_SUN_SYM: return HRD_CPLX6;
            case HRD_SUN_ASYM: return HRD_CPLX3;
            default: return -1;
        }
    }
    if (nc == 4) {
        switch (kind) {
            case HRD_SUN_FUND: return HRD_CPLX4;
            case HRD_SUN_ADJ: return HRD_REAL15;
            case HRD_SUN_SYM: return HRD_CPLX10;
            case HRD_SUN_ASYM: return HRD_CPLX6;
            default: return -1;
        }
    }
    return -1;
}

hrd_status hrd_represent_sun(const hrd_lattice *lat, int nc, hrd_sun_rep kind, const void *U_fund, void *U_rep,
                             void *stream)
{
    HRD_TRY(check_lattice(lat));
    const int out = hrd_sun_rep_format(nc, kind);
    if (out < 0) return fail(HRD_EINVAL, "no link format for SU(%d) representation %d", nc, (int)kind);
    if (!U_fund || !U_rep) return fail(HRD_EINVAL, "NULL field pointer");
    const int in = nc == 3 ? HRD_CPLX3 : HRD_CPLX4;
    if (overlap(U_fund, gauge_bytes(lat, in, HRD_F64), U_rep, gauge_bytes(lat, out, HRD_F64)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_represent_sun(nc, (int)kind, g, U_fund, U_rep, (hipStream_t)stream),
                     "represent_sun launch");
}

hrd_status hrd_represent_backward_sun(const hrd_lattice *lat, int nc, hrd_sun_rep kind, const void *U_fund,
                                      const void *G_rep, void *G_fund, void *stream)
{
    HRD_TRY(check_lattice(lat));
    const int rf = hrd_sun_rep_format(nc, kind);
    if (rf < 0) return fail(HRD_EINVAL, "no link format for SU(%d) representation %d", nc, (int)kind);
    if (!U_fund || !G_rep || !G_fund) return fail(HRD_EINVAL, "NULL field pointer");
    const int in = nc == 3 ? HRD_CPLX3 : HRD_CPLX4;
    const size_t nf = gauge_bytes(lat, in, HRD_F64), nr = gauge_bytes(lat, rf, HRD_F64);
    if (overlap(G_fund, nf, U_fund, nf) || overlap(G_fund, nf, G_rep, nr))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_represent_backward_sun(nc, (int)kind, g, U_fund, G_rep, G_fund, (hipStream_t)stream),
                     "represent_backward_sun launch");
}

hrd_status hrd_represent_backward(const hrd_lattice *lat, const void *U_fund, const void *g_adj, void *G_fund,
                                  void *stream)
{
    HRD_TRY(check_lattice(lat));
    if (!U_fund || !g_adj || !G_fund) return fail(HRD_EINVAL, "NULL field pointer");
    const size_t nf = gauge_bytes(lat, HRD_FUND, HRD_F64), na = gauge_bytes(lat, HRD_ADJ, HRD_F64);
    if (overlap(G_fund, nf, U_fund, nf) || overlap(G_fund, nf, g_adj, na)) return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_represent_backward(g, U_fund, g_adj, G_fund, (hipStream_t)stream), "represent_backward launch");
}

hrd_status hrd_convert_gauge(const hrd_lattice *lat, hrd_rep rep, const void *U64, void *U32, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, HRD_F32));
    if (!U64 || !U32) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(U64, gauge_bytes(lat, rep, HRD_F64), U32, gauge_bytes(lat, rep, HRD_F32)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_convert_gauge(rep, g, U64, U32, (hipStream_t)stream), "convert_gauge launch");
}

hrd_status hrd_pack_spinor(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, hrd_sites sites, const void *psi_nat,
                           void *psi, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (sites < HRD_SITES_ALL || sites > HRD_SITES_ODD) return fail(HRD_EINVAL, "invalid site subset %d", (int)sites);
    if (!psi_nat || !psi) return fail(HRD_EINVAL, "NULL field pointer");
    const int np = sites == HRD_SITES_ALL ? 2 : 1;
    if (overlap(psi_nat, spinor_bytes(lat, rep, HRD_F64, 2), psi, spinor_bytes(lat, rep, prec, np)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_pack_spinor(rep, prec, sites, g, psi_nat, psi, false, (hipStream_t)stream), "pack_spinor launch");
}

hrd_status hrd_unpack_spinor(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, hrd_sites sites, const void *psi,
                             void *psi_nat, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (sites < HRD_SITES_ALL || sites > HRD_SITES_ODD) return fail(HRD_EINVAL, "invalid site subset %d", (int)sites);
    if (!psi_nat || !psi) return fail(HRD_EINVAL, "NULL field pointer");
    const int np = sites == HRD_SITES_ALL ? 2 : 1;
    if (overlap(psi_nat, spinor_bytes(lat, rep, HRD_F64, 2), psi, spinor_bytes(lat, rep, prec, np)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_pack_spinor(rep, prec, sites, g, psi_nat, const_cast<void *>(psi), true, (hipStream_t)stream),
                     "unpack_spinor launch");
}

hrd_status hrd_convert_spinor(const hrd_lattice *lat, hrd_rep rep, int nparity, int to_f32, const void *in, void *out,
                              void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, HRD_F64));
    if (nparity != 1 && nparity != 2) return fail(HRD_EINVAL, "nparity must be 1 or 2");
    if (!in || !out) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(in, spinor_bytes(lat, rep, to_f32 ? HRD_F64 : HRD_F32, nparity), out,
                spinor_bytes(lat, rep, to_f32 ? HRD_F32 : HRD_F64, nparity)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_convert_spinor(g.Vh, nparity, ncomp_of(rep), to_f32 != 0, in, out, (hipStream_t)stream),
                     "convert_spinor launch");
}

hrd_status hrd_convert_spinor_prec(const hrd_lattice *lat, hrd_rep rep, int nparity, hrd_prec prec_in,
                                   hrd_prec prec_out, const void *in, void *out, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec_any(rep, prec_in));
    HRD_TRY(check_rep_prec_any(rep, prec_out));
    if (nparity != 1 && nparity != 2) return fail(HRD_EINVAL, "nparity must be 1 or 2");
    if (!in || !out) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(in, spinor_bytes(lat, rep, prec_in, nparity), out, spinor_bytes(lat, rep, prec_out, nparity)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_convert_spinor_prec(rep, g.Vh, nparity, prec_in, prec_out, in, out, (hipStream_t)stream),
                     "convert_spinor_prec launch");
}

hrd_status hrd_convert_gauge_prec(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec_out, const void *U64,
                                  void *U_out, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec_any(rep, prec_out));
    if (prec_out == HRD_F64) return fail(HRD_EINVAL, "prec_out must be HRD_F32 or HRD_F16");
    if (!U64 || !U_out) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(U64, gauge_bytes(lat, rep, HRD_F64), U_out, gauge_bytes(lat, rep, prec_out)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    const hipStream_t st = (hipStream_t)stream;
    return check_hip(prec_out == HRD_F32 ? launch_convert_gauge(rep, g, U64, U_out, st)
                                         : launch_convert_gauge_h16(rep, g, U64, U_out, st),
                     "convert_gauge_prec launch");
}

size_t hrd_dirac_workspace_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, hrd_parity parity)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec_any(rep, prec) != HRD_OK) return 0;
    return parity == HRD_EO ? spinor_bytes(lat, rep, prec, 1) : 0;
}

hrd_status hrd_dirac_apply(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, const void *psi,
                           void *out, double m0, hrd_parity parity, int dagger, void *work, void *stream)
{
    return hrd::dirac_apply_checked(lat, rep, prec, U, psi, out, m0, parity, dagger, work, stream);
}

}  // extern "C"

namespace hrd {

hrd_status dirac_apply_checked(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, const void *psi,
                               void *out, double m0, hrd_parity parity, int dagger, void *work, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec_any(rep, prec));
    if (parity < HRD_FULL || parity > HRD_HOP_OE) return fail(HRD_EINVAL, "invalid parity mode %d", (int)parity);
    if (!U || !psi || !out) return fail(HRD_EINVAL, "NULL field pointer");
    if (!std::isfinite(m0) || 4.0 + m0 == 0.0) return fail(HRD_EINVAL, "m0 = %g is not finite or makes 4 + m0 zero", m0);
    const int np = parity == HRD_FULL ? 2 : 1;
    const size_t sb = spinor_bytes(lat, rep, prec, np);
    const size_t ub = gauge_bytes(lat, rep, prec);
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub)) return fail(HRD_EALIAS, "output overlaps an input");
    if (parity == HRD_EO) {
        if (!work) return fail(HRD_EINVAL, "HRD_EO needs a workspace of hrd_dirac_workspace_bytes bytes");
        const size_t wb = spinor_bytes(lat, rep, prec, 1);
        if (overlap(work, wb, psi, sb) || overlap(work, wb, out, sb) || overlap(work, wb, U, ub))
            return fail(HRD_EALIAS, "workspace overlaps a field");
    }
    const Geom g = make_geom(lat->dims);
    const hipStream_t st = (hipStream_t)stream;
    const bool dag = dagger != 0;
    hipError_t e = hipSuccess;
    switch (parity) {
        case HRD_FULL: e = apply_full(rep, prec, g, U, psi, out, m0, dag, st); break;
        case HRD_EO: e = apply_dhat(rep, prec, g, U, psi, out, work, m0, dag, nullptr, st); break;
        case HRD_HOP_EO: e = apply_hop_block(rep, prec, g, U, psi, out, 0, dag, st); break;
        case HRD_HOP_OE: e = apply_hop_block(rep, prec, g, U, psi, out, 1, dag, st); break;
    }
    return check_hip(e, "dirac_apply launch");
}

}  // namespace hrd

extern "C" {

size_t hrd_clover_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec(rep, prec) != HRD_OK || !clover_capable(rep)) return 0;
    return clover_bytes(lat, rep, prec);
}

hrd_status hrd_clover_build(const hrd_lattice *lat, hrd_rep rep, hrd_clover_kind kind, const void *U64, double csw,
                            double m0, void *M64, void *Minv64, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_clover_format(rep, "hrd_clover_build"));
    HRD_TRY(check_rep_prec(rep, HRD_F64));
    if (kind != HRD_CLOVER_SW && kind != HRD_CLOVER_EXP) return fail(HRD_EINVAL, "invalid clover kind %d", (int)kind);
    if (!U64 || !M64 || !Minv64) return fail(HRD_EINVAL, "NULL field pointer");
    if (!std::isfinite(csw) || !std::isfinite(m0)) return fail(HRD_EINVAL, "csw and m0 must be finite");
    const size_t cb = clover_bytes(lat, rep, HRD_F64);
    const size_t ub = gauge_bytes(lat, rep, HRD_F64);
    if (overlap(M64, cb, Minv64, cb) || overlap(M64, cb, U64, ub) || overlap(Minv64, cb, U64, ub))
        return fail(HRD_EALIAS, "clover outputs overlap each other or the gauge field");
    const Geom g = make_geom(lat->dims);
    if (4.0 + m0 == 0.0) return fail(HRD_EINVAL, "m0 = -4 makes the mass term zero");
    return check_hip(launch_clover_build(rep, kind == HRD_CLOVER_EXP, g, U64, csw, 4.0 + m0, M64, Minv64,
                                         (hipStream_t)stream),
                     "clover_build launch");
}

hrd_status hrd_convert_clover(const hrd_lattice *lat, hrd_rep rep, const void *C64, void *C32, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_clover_format(rep, "hrd_convert_clover"));
    HRD_TRY(check_rep_prec(rep, HRD_F64));
    if (!C64 || !C32) return fail(HRD_EINVAL, "NULL field pointer");
    if (overlap(C64, clover_bytes(lat, rep, HRD_F64), C32, clover_bytes(lat, rep, HRD_F32)))
        return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_convert_clover(rep, g, C64, C32, (hipStream_t)stream), "convert_clover launch");
}

hrd_status hrd_unpack_clover(const hrd_lattice *lat, hrd_rep rep, const void *C64, void *C_nat, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_clover_format(rep, "hrd_unpack_clover"));
    HRD_TRY(check_rep_prec(rep, HRD_F64));
    if (!C64 || !C_nat) return fail(HRD_EINVAL, "NULL field pointer");
    const size_t cb = clover_bytes(lat, rep, HRD_F64);
    if (overlap(C64, cb, C_nat, 4 * cb)) return fail(HRD_EALIAS, "output overlaps input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_unpack_clover(rep, g, C64, C_nat, (hipStream_t)stream), "unpack_clover launch");
}

hrd_status hrd_dirac_apply_clover(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, const void *M,
                                  const void *Minv, const void *psi, void *out, hrd_parity parity, int dagger,
                                  void *work, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_clover_format(rep, "hrd_dirac_apply_clover"));
    HRD_TRY(check_rep_prec_any(rep, prec));
    if (parity != HRD_FULL && parity != HRD_EO)
        return fail(HRD_EINVAL, "clover operator supports HRD_FULL and HRD_EO (hop blocks are those of hrd_dirac_apply)");
    if (!U || !M || !psi || !out) return fail(HRD_EINVAL, "NULL field pointer");
    if (parity == HRD_EO && !Minv) return fail(HRD_EINVAL, "HRD_EO needs the inverse clover field");
    const int np = parity == HRD_FULL ? 2 : 1;
    const size_t sb = spinor_bytes(lat, rep, prec, np);
    const size_t ub = gauge_bytes(lat, rep, prec);
    const size_t cb = clover_bytes(lat, rep, prec == HRD_F16 ? HRD_F32 : prec);
    if (overlap(out, sb, psi, sb) || overlap(out, sb, U, ub) || overlap(out, sb, M, cb) ||
        overlap(out, sb, Minv, cb))
        return fail(HRD_EALIAS, "output overlaps an input");
    if (parity == HRD_EO) {
        if (!work) return fail(HRD_EINVAL, "HRD_EO needs a workspace of hrd_dirac_workspace_bytes bytes");
        const size_t wb = spinor_bytes(lat, rep, prec, 1);
        if (overlap(work, wb, psi, sb) || overlap(work, wb, out, sb) || overlap(work, wb, U, ub) ||
            overlap(work, wb, M, cb) || overlap(work, wb, Minv, cb))
            return fail(HRD_EALIAS, "workspace overlaps a field");
    }
    const Geom g = make_geom(lat->dims);
    const hipStream_t st = (hipStream_t)stream;
    const CloverRef cl{M, Minv};
    hipError_t e = parity == HRD_FULL ? apply_full(rep, prec, g, U, psi, out, 0.0, dagger != 0, st, &cl)
                                      : apply_dhat(rep, prec, g, U, psi, out, work, 0.0, dagger != 0, nullptr, st, &cl);
    return check_hip(e, "dirac_apply_clover launch");
}

size_t hrd_blas_workspace_bytes(void) { return sizeof(double) * (2 * kRedBlocks + 8); }

static hrd_status blas_common(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity, void *work)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (nparity != 1 && nparity != 2) return fail(HRD_EINVAL, "nparity must be 1 or 2");
    if (!work) return fail(HRD_EINVAL, "NULL workspace");
    return HRD_OK;
}

static hrd_status finish_reduction(double *partials, int ncol, double *result, hipStream_t st)
{
    double *sums = partials + 2 * kRedBlocks;
    HRD_TRY(check_hip(launch_finalize(partials, kRedBlocks, ncol, sums, st), "finalize launch"));
    HRD_TRY(check_hip(hipMemcpyAsync(result, sums, sizeof(double) * ncol, hipMemcpyDeviceToHost, st), "hipMemcpyAsync"));
    return check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
}

hrd_status hrd_blas_dot(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity, const void *a, const void *b,
                        double *result, void *work, void *stream)
{
    HRD_TRY(blas_common(lat, rep, prec, nparity, work));
    if (!a || !b || !result) return fail(HRD_EINVAL, "NULL pointer");
    const size_t n16 = spinor_bytes(lat, rep, prec, nparity) / 16;
    const hipStream_t st = (hipStream_t)stream;
    double *parts = (double *)work;
    HRD_TRY(check_hip(launch_dot_partials(prec, n16, a, b, parts, st), "dot launch"));
    return finish_reduction(parts, 2, result, st);
}

hrd_status hrd_blas_norm2(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity, const void *a,
                          double *result, void *work, void *stream)
{
    HRD_TRY(blas_common(lat, rep, prec, nparity, work));
    if (!a || !result) return fail(HRD_EINVAL, "NULL pointer");
    const size_t n16 = spinor_bytes(lat, rep, prec, nparity) / 16;
    const hipStream_t st = (hipStream_t)stream;
    double *parts = (double *)work;
    HRD_TRY(check_hip(launch_norm_partials(prec, n16, a, parts, st), "norm launch"));
    return finish_reduction(parts, 1, result, st);
}

hrd_status hrd_blas_axpy(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity, double a_re, double a_im,
                         const void *x, void *y, double *result, void *work, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (nparity != 1 && nparity != 2) return fail(HRD_EINVAL, "nparity must be 1 or 2");
    if (!x || !y) return fail(HRD_EINVAL, "NULL pointer");
    if (result && !work) return fail(HRD_EINVAL, "a fused norm needs a workspace");
    const size_t bytes = spinor_bytes(lat, rep, prec, nparity);
    if (overlap(x, bytes, y, bytes) && x != y) return fail(HRD_EALIAS, "x and y partially overlap");
    const size_t n16 = bytes / 16;
    const hipStream_t st = (hipStream_t)stream;
    double *parts = result ? (double *)work : nullptr;
    HRD_TRY(check_hip(launch_axpy(prec, n16, a_re, a_im, x, y, parts, st), "axpy launch"));
    if (!result) return HRD_OK;
    return finish_reduction(parts, 1, result, st);
}

hrd_status hrd_blas_xpay(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, int nparity, const void *x, double a_re,
                         double a_im, void *y, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (nparity != 1 && nparity != 2) return fail(HRD_EINVAL, "nparity must be 1 or 2");
    if (!x || !y) return fail(HRD_EINVAL, "NULL pointer");
    const size_t bytes = spinor_bytes(lat, rep, prec, nparity);
    if (overlap(x, bytes, y, bytes) && x != y) return fail(HRD_EALIAS, "x and y partially overlap");
    return check_hip(launch_xpay(prec, bytes / 16, x, a_re, a_im, y, (hipStream_t)stream), "xpay launch");
}

size_t hrd_cg_workspace_bytes(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec(rep, HRD_F64) != HRD_OK) return 0;
    if (mode != HRD_CG_F64 && mode != HRD_CG_MIXED && mode != HRD_CG_MIXED16) return 0;
    return carve_cg(lat, rep, mode, nullptr, nullptr);
}

// CG on D^+ D^ x = b (Wilson, or clover when cl64 is given; the mixed mode
// then also needs cl32).
static hrd_status cg_run(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode, const void *U64, const void *U32,
                         const CloverRef *cl64, const CloverRef *cl32, const void *b, void *x, double m0, double tol,
                         int maxiter, double delta, void *work, size_t work_bytes, hrd_cg_info *info, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    hrd_cg_info inf{};
    auto finish = [&](hrd_status s) {
        inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return s;
    };
    {
        hrd_status s = check_lattice(lat);
        if (s == HRD_OK) s = check_rep_prec(rep, HRD_F64);
        if (s != HRD_OK) return finish(s);
    }
    if (mode != HRD_CG_F64 && mode != HRD_CG_MIXED && mode != HRD_CG_MIXED16)
        return finish(fail(HRD_EINVAL, "invalid CG mode %d", (int)mode));
    if (!U64 || !b || !x || !work) return finish(fail(HRD_EINVAL, "NULL pointer"));
    if (mode != HRD_CG_F64 && !U32)
        return finish(fail(HRD_EINVAL, "mixed CG needs the reduced-precision gauge field (FP32 or F16)"));
    if (!cl64 && (!std::isfinite(m0) || 4.0 + m0 == 0.0)) return finish(fail(HRD_EINVAL, "invalid m0 %g", m0));
    if (cl64 && !clover_capable(rep)) return finish(check_clover_format(rep, "hrd_cg_solve_clover"));
    if (cl64 && (!cl64->M || !cl64->Minv)) return finish(fail(HRD_EINVAL, "NULL FP64 clover field"));
    if (cl64 && mode != HRD_CG_F64 && (!cl32 || !cl32->M || !cl32->Minv))
        return finish(fail(HRD_EINVAL, "mixed CG needs the FP32 clover fields"));
    if (!(tol > 0.0) || !std::isfinite(tol)) return finish(fail(HRD_EINVAL, "tol must be positive"));
    if (maxiter < 0) return finish(fail(HRD_EINVAL, "maxiter must be >= 0"));
    const size_t need = carve_cg(lat, rep, mode, nullptr, nullptr);
    if (work_bytes < need) return finish(fail(HRD_ESIZE, "workspace %zu < %zu bytes", work_bytes, need));
    const size_t h64 = spinor_bytes(lat, rep, HRD_F64, 1);
    if (overlap(x, h64, b, h64)) return finish(fail(HRD_EALIAS, "x overlaps b"));
    if (overlap(work, need, x, h64) || overlap(work, need, b, h64) ||
        overlap(work, need, U64, gauge_bytes(lat, rep, HRD_F64)))
        return finish(fail(HRD_EALIAS, "workspace overlaps a field"));
    if (cl64) {
        const size_t c64 = clover_bytes(lat, rep, HRD_F64), c32 = clover_bytes(lat, rep, HRD_F32);
        bool bad = overlap(work, need, cl64->M, c64) || overlap(work, need, cl64->Minv, c64) ||
                   overlap(x, h64, cl64->M, c64) || overlap(x, h64, cl64->Minv, c64);
        if (mode != HRD_CG_F64)
            bad = bad || overlap(work, need, cl32->M, c32) || overlap(work, need, cl32->Minv, c32) ||
                  overlap(x, h64, cl32->M, c32) || overlap(x, h64, cl32->Minv, c32);
        if (bad) return finish(fail(HRD_EALIAS, "a clover field overlaps x or the workspace"));
    }
    if (delta <= 0.0) delta = mode == HRD_CG_MIXED16 ? kDeltaMixed16 : kDeltaMixed;

    CgBuffers w;
    carve_cg(lat, rep, mode, work, &w);
    const Geom g = make_geom(lat->dims);
    const hipStream_t st = (hipStream_t)stream;
    const int nc = ncomp_of(rep);
    const size_t n64 = h64 / 16;
    // ||.||^2 partials written by one operator stage of the iteration
    const int hb = hop_partials(rep, mode == HRD_CG_F64 ? HRD_F64 : mode == HRD_CG_MIXED16 ? HRD_F16 : HRD_F32, g);
    double sc[S_COUNT];

#define CG_HIP(expr, what)                                        \
    do {                                                          \
        hrd_status s_ = check_hip((expr), what);                  \
        if (s_ != HRD_OK) return finish(s_);                      \
    } while (0)

    // ||b||^2
    CG_HIP(launch_zero(sizeof(double) * S_COUNT, w.sc, st), "zero");
    CG_HIP(launch_norm_partials(HRD_F64, n64, b, w.partials, st), "norm(b)");
    CG_HIP(launch_finalize(w.partials, kRedBlocks, 1, w.sc + S_BB, st), "finalize");
    {
        hrd_status s = read_scalars(w.sc, sc, st);
        if (s != HRD_OK) return finish(s);
    }
    const double bb = sc[S_BB];
    if (!std::isfinite(bb)) return finish(fail(HRD_EBREAKDOWN, "source has non-finite entries"));
    if (bb == 0.0) {
        CG_HIP(launch_zero(h64, x, st), "zero x");
        CG_HIP(hipStreamSynchronize(st), "sync");
        return finish(HRD_OK);
    }
    const double bnorm = std::sqrt(bb);
    const double target = tol * bnorm;

    // r = b - A x (FP64), rr = ||r||^2
    auto true_residual = [&](void) -> hrd_status {
        hipError_t e = apply_dhat(rep, HRD_F64, g, U64, x, w.q64, w.t64, m0, false, nullptr, st, cl64);
        if (e == hipSuccess) e = apply_dhat(rep, HRD_F64, g, U64, w.q64, w.Ap64, w.t64, m0, true, nullptr, st, cl64);
        if (e == hipSuccess) {
            if (mode == HRD_CG_F64) e = launch_cg_residual64(n64, b, w.Ap64, w.r64, w.partials, st);
            else e = launch_cg_residual_mixed(g.Vh, nc, b, w.Ap64, w.r64, w.r32, w.partials, st);
        }
        if (e == hipSuccess) e = launch_finalize(w.partials, kRedBlocks, 1, w.sc + S_RR, st);
        hrd_status s = check_hip(e, "true residual");
        if (s != HRD_OK) return s;
        return read_scalars(w.sc, sc, st);
    };

    {
        hrd_status s = true_residual();
        if (s != HRD_OK) return finish(s);
    }
    double rr = sc[S_RR];
    inf.true_rel_residual = std::sqrt(rr) / bnorm;
    inf.iterated_rel_residual = inf.true_rel_residual;
    if (!std::isfinite(rr)) return finish(fail(HRD_EBREAKDOWN, "initial residual is not finite"));
    if (std::sqrt(rr) <= target) return finish(HRD_OK);

    ScalarPipe pipe(st);
    {
        hrd_status s = pipe.init();
        if (s != HRD_OK) return finish(s);
    }
    int cur = 0;
    // Each iteration queues the next iteration's D^ p before the host waits
    // for this iteration's scalars: that stage only writes q, t and the
    // partials, which a restart or reliable update recomputes anyway.
    if (mode == HRD_CG_F64) {
        CG_HIP(launch_copy(h64, w.r64, w.p64, st), "copy");
        CG_HIP(apply_dhat(rep, HRD_F64, g, U64, w.p64, w.q64, w.t64, m0, false, w.partials, st, cl64), "D^ p");
        while (inf.iters < maxiter) {
            CG_HIP(launch_cg_alpha(w.partials, hb, w.sc, st), "alpha");
            CG_HIP(apply_dhat_dag_update_r(rep, HRD_F64, g, U64, w.q64, w.r64, w.t64, m0, w.sc, w.partials, st, cl64),
                   "r -= alpha D^+ q");
            CG_HIP(launch_cg_beta(w.partials, hb, w.sc, st), "beta");
            CG_HIP(launch_cg_update_xp64(n64, x, w.p64, w.r64, w.sc, st), "update x, p");
            inf.iters++;
            {
                hrd_status s = pipe.post(w.sc, cur);
                if (s != HRD_OK) return finish(s);
            }
            CG_HIP(apply_dhat(rep, HRD_F64, g, U64, w.p64, w.q64, w.t64, m0, false, w.partials, st, cl64), "D^ p");
            {
                hrd_status s = pipe.wait(cur, sc);
                if (s != HRD_OK) return finish(s);
            }
            cur ^= 1;
            if (sc[S_FLAG] != 0.0)
                return finish(fail(HRD_EBREAKDOWN, "CG breakdown at iteration %d (pAp = %g, rr = %g)", inf.iters,
                                   sc[S_PAP], sc[S_RRNEW]));
            rr = sc[S_RR];
            inf.iterated_rel_residual = std::sqrt(rr) / bnorm;
            if (std::sqrt(rr) <= target) {
                hrd_status s = true_residual();
                if (s != HRD_OK) return finish(s);
                rr = sc[S_RR];
                inf.true_rel_residual = std::sqrt(rr) / bnorm;
                if (std::sqrt(rr) <= target) return finish(HRD_OK);
                inf.restarts++;
                CG_HIP(launch_copy(h64, w.r64, w.p64, st), "copy");
                CG_HIP(apply_dhat(rep, HRD_F64, g, U64, w.p64, w.q64, w.t64, m0, false, w.partials, st, cl64), "D^ p");
            }
        }
        hrd_status s = true_residual();
        if (s != HRD_OK) return finish(s);
        inf.true_rel_residual = std::sqrt(sc[S_RR]) / bnorm;
        return finish(fail(HRD_ENOCONV, "CG did not converge in %d iterations (residual %g)", maxiter,
                           inf.true_rel_residual));
    }

    // mixed precision with reliable updates; the operator's fields are FP32
    // (MIXED) or F16 (MIXED16), the iterated residual r32 is FP32 in both.
    // The search directions cycle through a ring of kPRing slots; slots
    // 0 .. j-1 hold directions whose alpha p is not yet in x, which is brought
    // up to date when the ring is full, before each reliable update and at
    // the end (the same FP64 sums, in the same order, as updating x every
    // iteration).
    const int lp = mode == HRD_CG_MIXED16 ? HRD_F16 : HRD_F32;
    const size_t h32 = spinor_bytes(lat, rep, HRD_F32, 1);
    char *ring = static_cast<char *>(w.plo);
    auto slot = [&](int i) { return static_cast<void *>(ring + (size_t)i * w.pstride); };
    auto ring_op = [&](int m, int src, int dst, int beta_mode) {
        return launch_cg_ring(lp, g.Vh, nc, x, ring, w.pstride, m, src, dst, w.r32, w.sc, w.ahist, beta_mode, st);
    };
    if (lp == HRD_F32) CG_HIP(launch_copy(h32, w.r32, slot(0), st), "copy");
    else CG_HIP(launch_convert_spinor_prec(rep, g.Vh, 1, HRD_F32, HRD_F16, w.r32, slot(0), st), "p = r");
    int j = 0;
    CG_HIP(apply_dhat(rep, lp, g, U32, slot(0), w.qlo, w.tlo, m0, false, w.partials, st, cl32), "D^ p");
    double rmax = std::sqrt(rr);
    while (inf.iters < maxiter) {
        CG_HIP(launch_cg_alpha(w.partials, hb, w.sc, st, w.ahist + j), "alpha");
        CG_HIP(apply_dhat_dag_update_r(rep, lp, g, U32, w.qlo, w.r32, w.tlo, m0, w.sc, w.partials, st, cl32),
               "r -= alpha D^+ q");
        CG_HIP(launch_cg_beta(w.partials, hb, w.sc, st), "beta");
        inf.iters++;
        {
            hrd_status s = pipe.post(w.sc, cur);
            if (s != HRD_OK) return finish(s);
        }
        // next direction p = r + beta p_j (a full ring is folded into x first)
        const int nj = j + 1 < kPRing ? j + 1 : 0;
        CG_HIP(ring_op(nj == 0 ? kPRing : 0, j, nj, kBetaIter), "advance p");
        CG_HIP(apply_dhat(rep, lp, g, U32, slot(nj), w.qlo, w.tlo, m0, false, w.partials, st, cl32), "D^ p");
        {
            hrd_status s = pipe.wait(cur, sc);
            if (s != HRD_OK) return finish(s);
        }
        cur ^= 1;
        if (sc[S_FLAG] != 0.0)
            return finish(fail(HRD_EBREAKDOWN, "CG breakdown at iteration %d (pAp = %g, rr = %g)", inf.iters,
                               sc[S_PAP], sc[S_RRNEW]));
        const double rnew = std::sqrt(sc[S_RR]);
        inf.iterated_rel_residual = rnew / bnorm;
        rmax = std::max(rmax, rnew);
        if (rnew < delta * rmax || rnew <= target) {
            // x += alpha p over the pending slots 0 .. j; then r = b - A x in
            // FP64, r32 = f32(r), and p = r + (rr / rr_old) p_j into slot 0
            if (nj > 0) CG_HIP(ring_op(nj, 0, -1, kBetaIter), "update x");
            hrd_status s = true_residual();
            if (s != HRD_OK) return finish(s);
            inf.reliable_updates++;
            const double rt = std::sqrt(sc[S_RR]);
            inf.true_rel_residual = rt / bnorm;
            if (!std::isfinite(rt)) return finish(fail(HRD_EBREAKDOWN, "non-finite residual"));
            if (rt <= target) return finish(HRD_OK);
            // a true residual well above the iterated one means the
            // low-precision recurrence lost track before reaching the
            // threshold: restart the search direction from r and raise the
            // threshold for the following cycles
            const bool drifted = rt > 2.0 * rnew;
            if (drifted) {
                inf.restarts++;
                delta = std::min(0.5, 10.0 * delta);
            }
            rmax = rt;
            CG_HIP(ring_op(0, j, 0, drifted ? kBetaZero : kBetaRatio), "update p");
            j = 0;
            CG_HIP(apply_dhat(rep, lp, g, U32, slot(0), w.qlo, w.tlo, m0, false, w.partials, st, cl32), "D^ p");
        } else {
            j = nj;
        }
    }
    if (j > 0) CG_HIP(ring_op(j, 0, -1, kBetaIter), "update x");
    {
        hrd_status s = true_residual();
        if (s != HRD_OK) return finish(s);
    }
    inf.true_rel_residual = std::sqrt(sc[S_RR]) / bnorm;
    return finish(fail(HRD_ENOCONV, "mixed CG did not converge in %d iterations (residual %g)", maxiter,
                       inf.true_rel_residual));
#undef CG_HIP
}

hrd_status hrd_cg_solve(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode, const void *U64, const void *U32,
                        const void *b, void *x, double m0, double tol, int maxiter, double delta, void *work,
                        size_t work_bytes, hrd_cg_info *info, void *stream)
{
    return cg_run(lat, rep, mode, U64, U32, nullptr, nullptr, b, x, m0, tol, maxiter, delta, work, work_bytes, info,
                  stream);
}

hrd_status hrd_cg_solve_clover(const hrd_lattice *lat, hrd_rep rep, hrd_cg_mode mode, const void *U64,
                               const void *U32, const void *M64, const void *Minv64, const void *M32,
                               const void *Minv32, const void *b, void *x, double tol, int maxiter, double delta,
                               void *work, size_t work_bytes, hrd_cg_info *info, void *stream)
{
    const CloverRef c64{M64, Minv64}, c32{M32, Minv32};
    return cg_run(lat, rep, mode, U64, U32, &c64, &c32, b, x, 0.0, tol, maxiter, delta, work, work_bytes, info,
                  stream);
}

hrd_status hrd_dirac_force(const hrd_lattice *lat, hrd_rep rep, hrd_prec prec, const void *U, const void *X,
                           const void *Y, void *F, double scale, void *stream)
{
    (void)U;
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, prec));
    if (prec != HRD_F64) return fail(HRD_EINVAL, "the force is computed in FP64 only");
    if (!X || !Y || !F) return fail(HRD_EINVAL, "NULL field pointer");
    if (!std::isfinite(scale)) return fail(HRD_EINVAL, "scale is not finite");
    const size_t sb = spinor_bytes(lat, rep, HRD_F64, 2), fb = gauge_bytes(lat, base_rep(rep), HRD_F64);
    if (overlap(F, fb, X, sb) || overlap(F, fb, Y, sb)) return fail(HRD_EALIAS, "output overlaps an input");
    const Geom g = make_geom(lat->dims);
    return check_hip(launch_force(rep, g, X, Y, F, scale, (hipStream_t)stream), "force launch");
}

size_t hrd_action_force_workspace_bytes(const hrd_lattice *lat, hrd_rep rep)
{
    if (check_lattice(lat) != HRD_OK || check_rep_prec(rep, HRD_F64) != HRD_OK) return 0;
    return 2 * spinor_bytes(lat, rep, HRD_F64, 2) + 256;
}

hrd_status hrd_action_force(const hrd_lattice *lat, hrd_rep rep, const void *U, const void *xi, void *F, double m0,
                            double scale, void *work, size_t work_bytes, void *stream)
{
    HRD_TRY(check_lattice(lat));
    HRD_TRY(check_rep_prec(rep, HRD_F64));
    if (!U || !xi || !F || !work) return fail(HRD_EINVAL, "NULL pointer");
    if (!std::isfinite(m0) || 4.0 + m0 == 0.0) return fail(HRD_EINVAL, "invalid m0 %g", m0);
    if (!std::isfinite(scale)) return fail(HRD_EINVAL, "scale is not finite");
    const size_t need = 2 * spinor_bytes(lat, rep, HRD_F64, 2);
    if (work_bytes < need) return fail(HRD_ESIZE, "workspace %zu < %zu bytes", work_bytes, need);
    const size_t fb = gauge_bytes(lat, base_rep(rep), HRD_F64), h = spinor_bytes(lat, rep, HRD_F64, 1);
    const size_t ub = gauge_bytes(lat, rep, HRD_F64);
    if (overlap(F, fb, xi, h) || overlap(F, fb, U, ub) || overlap(work, need, F, fb) || overlap(work, need, xi, h) ||
        overlap(work, need, U, ub))
        return fail(HRD_EALIAS, "buffers overlap");
    const Geom g = make_geom(lat->dims);
    const hipStream_t st = (hipStream_t)stream;
    char *X = (char *)work;
    char *Y = X + 2 * h;
    // Y = (xi, D_oe xi) ; X = (eta, (D_eo)^+ eta) with eta = D^ xi
    hipError_t e = launch_copy(h, xi, Y, st);
    if (e == hipSuccess) e = apply_hop_block(rep, HRD_F64, g, U, xi, Y + h, 1, false, st);
    // eta = D^ xi, using the odd half of X as the temporary, then the odd half of X
    if (e == hipSuccess) e = apply_dhat(rep, HRD_F64, g, U, xi, X, X + h, m0, false, nullptr, st);
    if (e == hipSuccess) e = apply_hop_block(rep, HRD_F64, g, U, X, X + h, 1, true, st);
    if (e == hipSuccess) e = launch_force(rep, g, X, Y, F, scale * 2.0 / (4.0 + m0), st);
    return check_hip(e, "action force");
}

}  // extern "C"
