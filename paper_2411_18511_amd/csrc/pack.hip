// Field preparation: natural <-> packed layouts, the adjoint map of SU(2)
// links and its chain rule, and precision conversions.  The paper precomputes
// derived fields once per gauge update (Sec. 2.2); these kernels are that step
// for the representation and the FP32 copy.
#include <type_traits>

#include "kernels.h"

namespace hrd {

namespace {

template <int N, typename R>
__global__ __launch_bounds__(kBlock) void pack_spinor_kernel(Geom g, int p0, int np, const Cx<double> *nat,
                                                            char *packed, bool unpack)
{
    constexpr int NC = 4 * N;
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long)np * g.Vh) return;
    const int pp = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pp * g.Vh);
    const int p = p0 + pp;
    const Site s = eo_site(g, idx, p);
    const size_t half = (size_t)g.Vh * NC * sizeof(Cx<R>);
    char *blk = packed + (size_t)pp * half;
    Cx<double> *site_nat = const_cast<Cx<double> *>(nat) + (size_t)s.lex * NC;
    Cx<R> c[NC];
    if (!unpack) {
#pragma unroll
        for (int k = 0; k < NC; k++) c[k] = Cx<R>{(R)site_nat[k].re, (R)site_nat[k].im};
        SpinorIO<R>::template store<NC>(blk, g.Vh, idx, c);
    } else {
        SpinorIO<R>::template load<NC>(blk, g.Vh, idx, c);
#pragma unroll
        for (int k = 0; k < NC; k++) site_nat[k] = Cx<double>{(double)c[k].re, (double)c[k].im};
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void pack_gauge_fund_kernel(Geom g, Cx<double> *nat, void *packed,
                                                                bool unpack)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const long r = t - (long)mu * V;
    const int p = (int)(r / g.Vh);
    const int idx = (int)(r - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    Cx<double> *e = nat + ((size_t)mu * V + s.lex) * 4;
    using IO = LinkIO<HRD_FUND, R>;
    if (!unpack) {
        typename IO::Link l;
#pragma unroll
        for (int k = 0; k < 4; k++) l.u[k >> 1][k & 1] = Cx<R>{(R)e[k].re, (R)e[k].im};
        IO::store(packed, g.Vh, p, mu, idx, l);
    } else {
        const auto l = IO::load(packed, g.Vh, p, mu, idx);
#pragma unroll
        for (int k = 0; k < 4; k++) e[k] = Cx<double>{(double)l.u[k >> 1][k & 1].re, (double)l.u[k >> 1][k & 1].im};
    }
}

// FUND_SU2 / ADJ_SU2: keep the first row of each natural fundamental link;
// unpacking returns the full matrix with the second row reconstructed.
template <typename R>
__global__ __launch_bounds__(kBlock) void pack_gauge_su2_kernel(Geom g, Cx<double> *nat, void *packed, bool unpack)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const long r = t - (long)mu * V;
    const int p = (int)(r / g.Vh);
    const int idx = (int)(r - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    Cx<double> *e = nat + ((size_t)mu * V + s.lex) * 4;
    if (!unpack) {
        const Su2Row<R> row{{(R)e[0].re, (R)e[0].im}, {(R)e[1].re, (R)e[1].im}};
        RowIO<R>::store(packed, g.Vh, p, mu, idx, row);
    } else {
        const Su2Row<R> row = RowIO<R>::load(packed, g.Vh, p, mu, idx);
        e[0] = Cx<double>{(double)row.a.re, (double)row.a.im};
        e[1] = Cx<double>{(double)row.b.re, (double)row.b.im};
        e[2] = Cx<double>{-(double)row.b.re, (double)row.b.im};
        e[3] = Cx<double>{(double)row.a.re, -(double)row.a.im};
    }
}

__global__ __launch_bounds__(kBlock) void convert_gauge_su2_kernel(Geom g, const void *U64, void *U32)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    const Su2Row<double> a = RowIO<double>::load(U64, g.Vh, p, mu, idx);
    const Su2Row<float> b{{(float)a.a.re, (float)a.a.im}, {(float)a.b.re, (float)a.b.im}};
    RowIO<float>::store(U32, g.Vh, p, mu, idx, b);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void pack_gauge_adj_kernel(Geom g, double *nat, void *packed, bool unpack)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const long r = t - (long)mu * V;
    const int p = (int)(r / g.Vh);
    const int idx = (int)(r - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    double *e = nat + ((size_t)mu * V + s.lex) * 9;
    using IO = LinkIO<HRD_ADJ, R>;
    if (!unpack) {
        typename IO::Link l;
#pragma unroll
        for (int k = 0; k < 9; k++) l.r[k / 3][k % 3] = (R)e[k];
        IO::store(packed, g.Vh, p, mu, idx, l);
    } else {
        const auto l = IO::load(packed, g.Vh, p, mu, idx);
#pragma unroll
        for (int k = 0; k < 9; k++) e[k] = (double)l.r[k / 3][k % 3];
    }
}

// 2x2 complex helpers for the adjoint map
struct M2 {
    Cx<double> m[2][2];
};

__device__ __forceinline__ M2 mm(const M2 &a, const M2 &b)
{
    M2 c;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) c.m[i][j] = cfma(a.m[i][1], b.m[1][j], cmul(a.m[i][0], b.m[0][j]));
    return c;
}

__device__ __forceinline__ M2 dagger(const M2 &a)
{
    M2 c;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) c.m[i][j] = Cx<double>{a.m[j][i].re, -a.m[j][i].im};
    return c;
}

__device__ __forceinline__ M2 pauli(int a)
{
    M2 s;
    const Cx<double> z{0, 0}, one{1, 0}, mone{-1, 0}, pi{0, 1}, mi{0, -1};
    if (a == 0) {
        s.m[0][0] = z; s.m[0][1] = one; s.m[1][0] = one; s.m[1][1] = z;
    } else if (a == 1) {
        s.m[0][0] = z; s.m[0][1] = mi; s.m[1][0] = pi; s.m[1][1] = z;
    } else {
        s.m[0][0] = one; s.m[0][1] = z; s.m[1][0] = z; s.m[1][1] = mone;
    }
    return s;
}

// real part of tr(s_a X): s1 -> X01 + X10, s2 -> i (X01 - X10), s3 -> X00 - X11
__device__ __forceinline__ double re_tr_pauli(int a, const M2 &X)
{
    if (a == 0) return X.m[0][1].re + X.m[1][0].re;
    if (a == 1) return -X.m[0][1].im + X.m[1][0].im;
    return X.m[0][0].re - X.m[1][1].re;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void represent_kernel(Geom g, const void *Uf, void *Ua)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int pm = (int)(t / g.Vh);  // 4 p + mu
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    const auto u = LinkIO<HRD_FUND, double>::load(Uf, g.Vh, p, mu, idx);
    M2 U, Ud;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) U.m[i][j] = u.u[i][j];
    Ud = dagger(U);
    typename LinkIO<HRD_ADJ, R>::Link l;
#pragma unroll
    for (int b = 0; b < 3; b++) {
        const M2 Mb = mm(mm(U, pauli(b)), Ud);  // U s_b U^+
#pragma unroll
        for (int a = 0; a < 3; a++) l.r[a][b] = (R)(0.5 * re_tr_pauli(a, Mb));
    }
    LinkIO<HRD_ADJ, R>::store(Ua, g.Vh, p, mu, idx, l);
}

// G = sum_ab g_ab s_a U s_b  (chain rule of R(U) in the dL/dReU + i dL/dImU convention)
__global__ __launch_bounds__(kBlock) void represent_backward_kernel(Geom g, const void *Uf, const void *ga, void *Gf)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    const auto u = LinkIO<HRD_FUND, double>::load(Uf, g.Vh, p, mu, idx);
    const auto ad = LinkIO<HRD_ADJ, double>::load(ga, g.Vh, p, mu, idx);
    M2 U;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) U.m[i][j] = u.u[i][j];
    M2 acc;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc.m[i][j] = Cx<double>{0, 0};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const M2 sU = mm(pauli(a), U);
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const M2 t2 = mm(sU, pauli(b));
            const double w = ad.r[a][b];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    acc.m[i][j] = Cx<double>{acc.m[i][j].re + w * t2.m[i][j].re, acc.m[i][j].im + w * t2.m[i][j].im};
        }
    }
    FundLink<double> out;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) out.u[i][j] = acc.m[i][j];
    LinkIO<HRD_FUND, double>::store(Gf, g.Vh, p, mu, idx, out);
}

template <int REP>
__global__ __launch_bounds__(kBlock) void convert_gauge_kernel(Geom g, const void *U64, void *U32)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    const auto a = LinkIO<REP, double>::load(U64, g.Vh, p, mu, idx);
    typename LinkIO<REP, float>::Link b;
    if constexpr (REP == HRD_FUND) {
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) b.u[i][j] = Cx<float>{(float)a.u[i][j].re, (float)a.u[i][j].im};
    } else {
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) b.r[i][j] = (float)a.r[i][j];
    }
    LinkIO<REP, float>::store(U32, g.Vh, p, mu, idx, b);
}

// F64 plane k (complex128) <-> F32 plane k/2 slot k%2; one thread per
// (parity block, F32 plane, site).
__global__ __launch_bounds__(kBlock) void convert_spinor_kernel(int Vh, int nparity, int ncomp, bool to_f32,
                                                               const void *in, void *out)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const int npl = ncomp / 2;
    if (t >= (long)nparity * npl * Vh) return;
    const int blk = (int)(t / ((long)npl * Vh));
    const long r = t - (long)blk * npl * Vh;
    const MixOff o = mix_off(r, Vh, npl);
    char *d = static_cast<char *>(to_f32 ? const_cast<void *>(in) : out) + (size_t)blk * ncomp * Vh * 16;
    char *f = static_cast<char *>(to_f32 ? out : const_cast<void *>(in)) + (size_t)blk * npl * Vh * 16;
    double2 *d0 = reinterpret_cast<double2 *>(d + o.f64a);
    double2 *d1 = reinterpret_cast<double2 *>(d + o.f64b);
    float4 *fv = reinterpret_cast<float4 *>(f + o.f32);
    if (to_f32) {
        const double2 a = *d0, b = *d1;
        *fv = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
    } else {
        const float4 v = *fv;
        *d0 = make_double2(v.x, v.y);
        *d1 = make_double2(v.z, v.w);
    }
}

// F64 links -> F16 links (binary16 of the FP32 rounding of each entry); one
// thread per (parity, direction, site).
template <int REP>
__global__ __launch_bounds__(kBlock) void convert_gauge_h16_kernel(Geom g, const void *U64, void *U16)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    if constexpr (is_su2_row(REP)) {
        RowIO<h16>::store(U16, g.Vh, p, mu, idx, RowIO<double>::load(U64, g.Vh, p, mu, idx));
    } else {
        LinkIO<REP, h16>::store(U16, g.Vh, p, mu, idx, LinkIO<REP, double>::load(U64, g.Vh, p, mu, idx));
    }
}

// Spinor storage conversion, one thread per site of each parity block: the
// input is read in its arithmetic type, rounded to the output's and stored
// (F16 output computes its site scale in FP32); F16 -> F64 is exact.
template <int NC, typename SI, typename SO>
__global__ __launch_bounds__(kBlock) void convert_spinor_site_kernel(int Vh, int nparity, size_t in_blk,
                                                                    size_t out_blk, const void *in, void *out)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long)nparity * Vh) return;
    const int blk = (int)(t / Vh);
    const int site = (int)(t - (long)blk * Vh);
    const char *src = reinterpret_cast<const char *>(in) + blk * in_blk;
    char *dst = reinterpret_cast<char *>(out) + blk * out_blk;
    using RO = typename Arith<SO>::type;
    Cx<RO> co[NC];
    if constexpr (std::is_same<SI, h16>::value && std::is_same<SO, double>::value) {
        SpinorIO<h16>::load_exact<NC>(src, Vh, site, co);
    } else {
        using RI = typename Arith<SI>::type;
        Cx<RI> ci[NC];
        SpinorIO<SI>::template load<NC>(src, Vh, site, ci);
#pragma unroll
        for (int k = 0; k < NC; k++) co[k] = Cx<RO>{(RO)ci[k].re, (RO)ci[k].im};
    }
    SpinorIO<SO>::template store<NC>(dst, Vh, site, co);
}

inline dim3 grid_for(long n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

namespace {

template <int N>
void pack_spinor_n(int prec, dim3 grid, hipStream_t st, const Geom &g, int p0, int np, const Cx<double> *n, char *pk,
                   bool unpack)
{
    if (prec == HRD_F64) hipLaunchKernelGGL((pack_spinor_kernel<N, double>), grid, dim3(kBlock), 0, st, g, p0, np, n, pk, unpack);
    else hipLaunchKernelGGL((pack_spinor_kernel<N, float>), grid, dim3(kBlock), 0, st, g, p0, np, n, pk, unpack);
}

}  // namespace

hipError_t launch_pack_spinor(int rep, int prec, int sites, const Geom &g, const void *nat, void *packed,
                              bool unpack, hipStream_t st)
{
    const int p0 = (sites == HRD_SITES_ODD) ? 1 : 0;
    const int np = (sites == HRD_SITES_ALL) ? 2 : 1;
    const dim3 grid = grid_for((long)np * g.Vh);
    const Cx<double> *n = reinterpret_cast<const Cx<double> *>(nat);
    char *pk = reinterpret_cast<char *>(packed);
    switch (ncolour(rep)) {
        case 2: pack_spinor_n<2>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        case 3: pack_spinor_n<3>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        case 4: pack_spinor_n<4>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        case 6: pack_spinor_n<6>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        case 8: pack_spinor_n<8>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        case 10: pack_spinor_n<10>(prec, grid, st, g, p0, np, n, pk, unpack); break;
        default: pack_spinor_n<15>(prec, grid, st, g, p0, np, n, pk, unpack); break;
    }
    return hipGetLastError();
}

hipError_t launch_pack_gauge(int rep, int prec, const Geom &g, const void *nat, void *packed, bool unpack,
                             hipStream_t st)
{
    if (is_dense(rep)) return launch_pack_gauge_dense(rep, prec, g, nat, packed, unpack, st);
    const dim3 grid = grid_for(8L * g.Vh);
    if (is_su2_row(rep)) {
        Cx<double> *n = reinterpret_cast<Cx<double> *>(const_cast<void *>(nat));
        if (prec == HRD_F64) hipLaunchKernelGGL((pack_gauge_su2_kernel<double>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
        else hipLaunchKernelGGL((pack_gauge_su2_kernel<float>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
    } else if (rep == HRD_FUND) {
        Cx<double> *n = reinterpret_cast<Cx<double> *>(const_cast<void *>(nat));
        if (prec == HRD_F64) hipLaunchKernelGGL((pack_gauge_fund_kernel<double>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
        else hipLaunchKernelGGL((pack_gauge_fund_kernel<float>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
    } else {
        double *n = reinterpret_cast<double *>(const_cast<void *>(nat));
        if (prec == HRD_F64) hipLaunchKernelGGL((pack_gauge_adj_kernel<double>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
        else hipLaunchKernelGGL((pack_gauge_adj_kernel<float>), grid, dim3(kBlock), 0, st, g, n, packed, unpack);
    }
    return hipGetLastError();
}

hipError_t launch_represent(int prec_out, const Geom &g, const void *Uf, void *Ua, hipStream_t st)
{
    const dim3 grid = grid_for(8L * g.Vh);
    if (prec_out == HRD_F64) hipLaunchKernelGGL((represent_kernel<double>), grid, dim3(kBlock), 0, st, g, Uf, Ua);
    else hipLaunchKernelGGL((represent_kernel<float>), grid, dim3(kBlock), 0, st, g, Uf, Ua);
    return hipGetLastError();
}

hipError_t launch_represent_backward(const Geom &g, const void *Uf, const void *ga, void *Gf, hipStream_t st)
{
    hipLaunchKernelGGL(represent_backward_kernel, grid_for(8L * g.Vh), dim3(kBlock), 0, st, g, Uf, ga, Gf);
    return hipGetLastError();
}

hipError_t launch_convert_gauge(int rep, const Geom &g, const void *U64, void *U32, hipStream_t st)
{
    if (is_dense(rep)) return launch_convert_gauge_dense(rep, HRD_F32, g, U64, U32, st);
    const dim3 grid = grid_for(8L * g.Vh);
    if (is_su2_row(rep)) hipLaunchKernelGGL(convert_gauge_su2_kernel, grid, dim3(kBlock), 0, st, g, U64, U32);
    else if (rep == HRD_FUND) hipLaunchKernelGGL((convert_gauge_kernel<HRD_FUND>), grid, dim3(kBlock), 0, st, g, U64, U32);
    else hipLaunchKernelGGL((convert_gauge_kernel<HRD_ADJ>), grid, dim3(kBlock), 0, st, g, U64, U32);
    return hipGetLastError();
}

hipError_t launch_convert_spinor(int Vh, int nparity, int ncomp, bool to_f32, const void *in, void *out,
                                 hipStream_t st)
{
    const long n = (long)nparity * (ncomp / 2) * Vh;
    hipLaunchKernelGGL(convert_spinor_kernel, grid_for(n), dim3(kBlock), 0, st, Vh, nparity, ncomp, to_f32, in, out);
    return hipGetLastError();
}

hipError_t launch_convert_gauge_h16(int rep, const Geom &g, const void *U64, void *U16, hipStream_t st)
{
    if (is_dense(rep)) return launch_convert_gauge_dense(rep, HRD_F16, g, U64, U16, st);
    const dim3 grid = grid_for(8L * g.Vh);
    switch (rep) {
        case HRD_FUND: hipLaunchKernelGGL((convert_gauge_h16_kernel<HRD_FUND>), grid, dim3(kBlock), 0, st, g, U64, U16); break;
        case HRD_ADJ: hipLaunchKernelGGL((convert_gauge_h16_kernel<HRD_ADJ>), grid, dim3(kBlock), 0, st, g, U64, U16); break;
        case HRD_FUND_SU2:
            hipLaunchKernelGGL((convert_gauge_h16_kernel<HRD_FUND_SU2>), grid, dim3(kBlock), 0, st, g, U64, U16);
            break;
        default:
            hipLaunchKernelGGL((convert_gauge_h16_kernel<HRD_ADJ_SU2>), grid, dim3(kBlock), 0, st, g, U64, U16);
            break;
    }
    return hipGetLastError();
}

namespace {

template <int NC, typename SI>
void convert_from(int prec_out, int Vh, int nparity, size_t ib, size_t ob, const void *in, void *out, hipStream_t st)
{
    const dim3 grid = grid_for((long)nparity * Vh);
    switch (prec_out) {
        case HRD_F64:
            hipLaunchKernelGGL((convert_spinor_site_kernel<NC, SI, double>), grid, dim3(kBlock), 0, st, Vh, nparity, ib,
                               ob, in, out);
            break;
        case HRD_F32:
            hipLaunchKernelGGL((convert_spinor_site_kernel<NC, SI, float>), grid, dim3(kBlock), 0, st, Vh, nparity, ib,
                               ob, in, out);
            break;
        default:
            hipLaunchKernelGGL((convert_spinor_site_kernel<NC, SI, h16>), grid, dim3(kBlock), 0, st, Vh, nparity, ib,
                               ob, in, out);
            break;
    }
}

template <int NC>
void convert_nc(int prec_in, int prec_out, int Vh, int nparity, size_t ib, size_t ob, const void *in, void *out,
                hipStream_t st)
{
    switch (prec_in) {
        case HRD_F64: convert_from<NC, double>(prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case HRD_F32: convert_from<NC, float>(prec_out, Vh, nparity, ib, ob, in, out, st); break;
        default: convert_from<NC, h16>(prec_out, Vh, nparity, ib, ob, in, out, st); break;
    }
}

}  // namespace

hipError_t launch_convert_spinor_prec(int rep, int Vh, int nparity, int prec_in, int prec_out, const void *in,
                                      void *out, hipStream_t st)
{
    const size_t ib = (size_t)Vh * spinor_site_bytes(rep, prec_in);
    const size_t ob = (size_t)Vh * spinor_site_bytes(rep, prec_out);
    if (prec_in == prec_out) return launch_copy(ib * nparity, in, out, st);
    switch (ncolour(rep)) {
        case 2: convert_nc<8>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case 3: convert_nc<12>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case 4: convert_nc<16>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case 6: convert_nc<24>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case 8: convert_nc<32>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        case 10: convert_nc<40>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
        default: convert_nc<60>(prec_in, prec_out, Vh, nparity, ib, ob, in, out, st); break;
    }
    return hipGetLastError();
}

}  // namespace hrd
