// Level-1 linear algebra on packed spinor fields and the fused vector stages
// of the conjugate-gradient solvers.  Fields are viewed as arrays of 16-byte
// elements (one complex128, or two complex64); the layouts of hrd.h keep
// complex pairs inside one element, so element-wise kernels and reductions do
// not need the site structure, except where FP64 and FP32 fields meet.
//
// Reductions: a fixed grid of kRedBlocks blocks walks the field with a
// grid-stride loop, each block writes its partial (wave64 butterfly + LDS),
// and one block sums the partials in a fixed order — bitwise reproducible,
// always accumulated in FP64.
#include "kernels.h"

namespace hrd {

namespace {

constexpr int kRedThreads = 256;

template <typename R>
struct Elem;
template <>
struct Elem<double> {
    static constexpr int C = 1;
    __device__ __forceinline__ static void load(const void *p, size_t i, Cx<double> (&c)[1])
    {
        const double2 v = reinterpret_cast<const double2 *>(p)[i];
        c[0] = {v.x, v.y};
    }
    __device__ __forceinline__ static void store(void *p, size_t i, const Cx<double> (&c)[1])
    {
        reinterpret_cast<double2 *>(p)[i] = make_double2(c[0].re, c[0].im);
    }
};
template <>
struct Elem<float> {
    static constexpr int C = 2;
    __device__ __forceinline__ static void load(const void *p, size_t i, Cx<float> (&c)[2])
    {
        const float4 v = reinterpret_cast<const float4 *>(p)[i];
        c[0] = {v.x, v.y};
        c[1] = {v.z, v.w};
    }
    __device__ __forceinline__ static void store(void *p, size_t i, const Cx<float> (&c)[2])
    {
        reinterpret_cast<float4 *>(p)[i] = make_float4(c[0].re, c[0].im, c[1].re, c[1].im);
    }
};

template <typename R>
__global__ __launch_bounds__(kRedThreads) void dot_kernel(size_t n, const void *a, const void *b, double *partials)
{
    constexpr int C = Elem<R>::C;
    double re = 0, im = 0;
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
        Cx<R> x[C], y[C];
        Elem<R>::load(a, i, x);
        Elem<R>::load(b, i, y);
#pragma unroll
        for (int k = 0; k < C; k++) {
            re += (double)x[k].re * y[k].re + (double)x[k].im * y[k].im;
            im += (double)x[k].re * y[k].im - (double)x[k].im * y[k].re;
        }
    }
    block_sum2<kRedThreads>(re, im);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

template <typename R>
__global__ __launch_bounds__(kRedThreads) void norm_kernel(size_t n, const void *a, double *partials)
{
    constexpr int C = Elem<R>::C;
    double s = 0;
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
        Cx<R> x[C];
        Elem<R>::load(a, i, x);
#pragma unroll
        for (int k = 0; k < C; k++) s += (double)x[k].re * x[k].re + (double)x[k].im * x[k].im;
    }
    s = block_sum<kRedThreads>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// y <- y + a x, optional ||y||^2 partials
template <typename R, bool NORM>
__global__ __launch_bounds__(kRedThreads) void axpy_kernel(size_t n, double ar, double ai, const void *x, void *y,
                                                          double *partials)
{
    constexpr int C = Elem<R>::C;
    const R cr = (R)ar, ci = (R)ai;
    double s = 0;
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
        Cx<R> u[C], v[C];
        Elem<R>::load(x, i, u);
        Elem<R>::load(y, i, v);
#pragma unroll
        for (int k = 0; k < C; k++) {
            v[k] = cfma(Cx<R>{cr, ci}, u[k], v[k]);
            if (NORM) s += (double)v[k].re * v[k].re + (double)v[k].im * v[k].im;
        }
        Elem<R>::store(y, i, v);
    }
    if constexpr (NORM) {
        s = block_sum<kRedThreads>(s);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

// y <- x + a y
template <typename R>
__global__ __launch_bounds__(kBlock) void xpay_kernel(size_t n, const void *x, double ar, double ai, void *y)
{
    constexpr int C = Elem<R>::C;
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    Cx<R> u[C], v[C];
    Elem<R>::load(x, i, u);
    Elem<R>::load(y, i, v);
#pragma unroll
    for (int k = 0; k < C; k++) v[k] = cfma(Cx<R>{(R)ar, (R)ai}, v[k], u[k]);
    Elem<R>::store(y, i, v);
}

constexpr int kFinThreads = 1024;

// Column sums of a [nblk][ncol] table, fixed order.
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(const double *partials, int nblk, int ncol, double *sums)
{
    for (int c = 0; c < ncol; c++) {
        double s = 0;
        for (int k = threadIdx.x; k < nblk; k += kFinThreads) s += partials[(size_t)k * ncol + c];
        s = block_sum<kFinThreads>(s);
        if (threadIdx.x == 0) sums[c] = s;
    }
}

__device__ __forceinline__ double fixed_sum(const double *partials, int nblk)
{
    double s = 0;
    for (int k = threadIdx.x; k < nblk; k += kFinThreads) s += partials[k];
    return block_sum<kFinThreads>(s);
}

__global__ __launch_bounds__(kFinThreads) void cg_alpha_kernel(const double *partials, int nblk, double *sc,
                                                                double *hist)
{
    const double pap = fixed_sum(partials, nblk);
    if (threadIdx.x == 0) {
        sc[S_PAP] = pap;
        double alpha = 0.0;
        if (!(pap > 0.0) || !isfinite(pap)) sc[S_FLAG] = 1.0;
        else alpha = sc[S_RR] / pap;
        sc[S_ALPHA] = alpha;
        if (hist) *hist = alpha;
    }
}

__global__ __launch_bounds__(kFinThreads) void cg_beta_kernel(const double *partials, int nblk, double *sc)
{
    const double rr = fixed_sum(partials, nblk);
    if (threadIdx.x == 0) {
        sc[S_RRNEW] = rr;
        if (!isfinite(rr)) {
            sc[S_FLAG] = 2.0;
            sc[S_BETA] = 0.0;
        } else {
            sc[S_BETA] = (sc[S_RR] > 0.0) ? rr / sc[S_RR] : 0.0;
        }
        sc[S_RROLD] = sc[S_RR];
        sc[S_RR] = rr;
    }
}

template <typename R>
__global__ __launch_bounds__(kRedThreads) void cg_update_r_kernel(size_t n, void *r, const void *Ap, const double *sc,
                                                                 double *partials)
{
    constexpr int C = Elem<R>::C;
    const R alpha = (R)sc[S_ALPHA];
    double s = 0;
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
        Cx<R> u[C], v[C];
        Elem<R>::load(r, i, u);
        Elem<R>::load(Ap, i, v);
#pragma unroll
        for (int k = 0; k < C; k++) {
            u[k] = Cx<R>{u[k].re - alpha * v[k].re, u[k].im - alpha * v[k].im};
            s += (double)u[k].re * u[k].re + (double)u[k].im * u[k].im;
        }
        Elem<R>::store(r, i, u);
    }
    s = block_sum<kRedThreads>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void cg_update_xp64_kernel(size_t n, void *x, void *p, const void *r, const double *sc)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double alpha = sc[S_ALPHA], beta = sc[S_BETA];
    double2 *X = reinterpret_cast<double2 *>(x);
    double2 *P = reinterpret_cast<double2 *>(p);
    const double2 rv = reinterpret_cast<const double2 *>(r)[i];
    const double2 pv = P[i];
    double2 xv = X[i];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    X[i] = xv;
    P[i] = make_double2(rv.x + beta * pv.x, rv.y + beta * pv.y);
}

// Mixed CG, FP32 search directions kept in a ring of kPRing slots, `stride`
// bytes apart.  Thread per (F32 plane q, site j); F64 planes 2q, 2q+1.
// MODE bit 1 (flush): x64 += alpha_s f64(p_s) for the slots s = 0 .. m-1 in
// order, alpha_s = ahist[s] — the same FP64 operations in the same order as
// updating x every iteration.  MODE bit 2 (advance): p_dst = r32 + beta p_src
// with beta chosen by ring_beta().
__device__ __forceinline__ float ring_beta(const double *sc, int beta_mode)
{
    if (beta_mode == kBetaRatio) return (float)(sc[S_RROLD] > 0.0 ? sc[S_RR] / sc[S_RROLD] : 0.0);
    if (beta_mode == kBetaZero) return 0.0f;
    return (float)sc[S_BETA];
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void cg_ring_f32_kernel(int Vh, int npl, void *x64, char *ring, size_t stride,
                                                             int m, int src, int dst, const void *r32,
                                                             const double *sc, const double *ahist, int beta_mode)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long)npl * Vh) return;
    const MixOff o = mix_off(t, Vh, npl);
    if constexpr ((MODE & 1) != 0) {
        double2 *X0 = reinterpret_cast<double2 *>(static_cast<char *>(x64) + o.f64a);
        double2 *X1 = reinterpret_cast<double2 *>(static_cast<char *>(x64) + o.f64b);
        double2 x0 = *X0, x1 = *X1;
#pragma unroll
        for (int s = 0; s < kPRing; s++) {
            if (s < m) {
                const double alpha = ahist[s];
                const float4 pv = *reinterpret_cast<const float4 *>(ring + (size_t)s * stride + o.f32);
                x0.x += alpha * (double)pv.x;
                x0.y += alpha * (double)pv.y;
                x1.x += alpha * (double)pv.z;
                x1.y += alpha * (double)pv.w;
            }
        }
        *X0 = x0;
        *X1 = x1;
    }
    if constexpr ((MODE & 2) != 0) {
        const float beta = ring_beta(sc, beta_mode);
        const float4 pv = *reinterpret_cast<const float4 *>(ring + (size_t)src * stride + o.f32);
        const float4 rv = *reinterpret_cast<const float4 *>(static_cast<const char *>(r32) + o.f32);
        *reinterpret_cast<float4 *>(ring + (size_t)dst * stride + o.f32) =
            make_float4(rv.x + beta * pv.x, rv.y + beta * pv.y, rv.z + beta * pv.z, rv.w + beta * pv.w);
    }
}

__global__ __launch_bounds__(kBlock) void cg_update_p32_kernel(size_t n, void *p32, const void *r32, const double *sc)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float beta = (float)(sc[S_RROLD] > 0.0 ? sc[S_RR] / sc[S_RROLD] : 0.0);
    float4 *P = reinterpret_cast<float4 *>(p32);
    const float4 pv = P[i];
    const float4 rv = reinterpret_cast<const float4 *>(r32)[i];
    P[i] = make_float4(rv.x + beta * pv.x, rv.y + beta * pv.y, rv.z + beta * pv.z, rv.w + beta * pv.w);
}

__global__ __launch_bounds__(kRedThreads) void cg_residual_mixed_kernel(int Vh, int npl, const void *b, const void *Ax,
                                                                       void *r64, void *r32, double *partials)
{
    const long n = (long)npl * Vh;
    double s = 0;
    for (long t = (long)blockIdx.x * kRedThreads + threadIdx.x; t < n; t += (long)gridDim.x * kRedThreads) {
        const MixOff o = mix_off(t, Vh, npl);
        auto d2 = [](const void *base, size_t off) {
            return *reinterpret_cast<const double2 *>(static_cast<const char *>(base) + off);
        };
        const double2 b0 = d2(b, o.f64a), b1 = d2(b, o.f64b);
        const double2 a0 = d2(Ax, o.f64a), a1 = d2(Ax, o.f64b);
        const double2 r0 = make_double2(b0.x - a0.x, b0.y - a0.y);
        const double2 r1 = make_double2(b1.x - a1.x, b1.y - a1.y);
        *reinterpret_cast<double2 *>(static_cast<char *>(r64) + o.f64a) = r0;
        *reinterpret_cast<double2 *>(static_cast<char *>(r64) + o.f64b) = r1;
        *reinterpret_cast<float4 *>(static_cast<char *>(r32) + o.f32) =
            make_float4((float)r0.x, (float)r0.y, (float)r1.x, (float)r1.y);
        s += r0.x * r0.x + r0.y * r0.y + r1.x * r1.x + r1.y * r1.y;
    }
    s = block_sum<kRedThreads>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void cg_residual64_kernel(size_t n, const void *b, const void *Ax, void *r,
                                                                   double *partials)
{
    double s = 0;
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kRedThreads) {
        const double2 bv = reinterpret_cast<const double2 *>(b)[i];
        const double2 av = reinterpret_cast<const double2 *>(Ax)[i];
        const double2 rv = make_double2(bv.x - av.x, bv.y - av.y);
        reinterpret_cast<double2 *>(r)[i] = rv;
        s += rv.x * rv.x + rv.y * rv.y;
    }
    s = block_sum<kRedThreads>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void copy16_kernel(size_t n, const float4 *src, float4 *dst)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void zero16_kernel(size_t n, float4 *dst)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

inline dim3 grid_for(size_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

hipError_t launch_dot_partials(int prec, size_t n16, const void *a, const void *b, double *partials, hipStream_t st)
{
    if (prec == HRD_F64) hipLaunchKernelGGL(dot_kernel<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, a, b, partials);
    else hipLaunchKernelGGL(dot_kernel<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, a, b, partials);
    return hipGetLastError();
}

hipError_t launch_norm_partials(int prec, size_t n16, const void *a, double *partials, hipStream_t st)
{
    if (prec == HRD_F64) hipLaunchKernelGGL(norm_kernel<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, a, partials);
    else hipLaunchKernelGGL(norm_kernel<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, a, partials);
    return hipGetLastError();
}

hipError_t launch_axpy(int prec, size_t n16, double ar, double ai, const void *x, void *y, double *partials,
                       hipStream_t st)
{
    const dim3 g(kRedBlocks), b(kRedThreads);
    if (prec == HRD_F64) {
        if (partials) hipLaunchKernelGGL((axpy_kernel<double, true>), g, b, 0, st, n16, ar, ai, x, y, partials);
        else hipLaunchKernelGGL((axpy_kernel<double, false>), g, b, 0, st, n16, ar, ai, x, y, partials);
    } else {
        if (partials) hipLaunchKernelGGL((axpy_kernel<float, true>), g, b, 0, st, n16, ar, ai, x, y, partials);
        else hipLaunchKernelGGL((axpy_kernel<float, false>), g, b, 0, st, n16, ar, ai, x, y, partials);
    }
    return hipGetLastError();
}

hipError_t launch_xpay(int prec, size_t n16, const void *x, double ar, double ai, void *y, hipStream_t st)
{
    if (prec == HRD_F64) hipLaunchKernelGGL(xpay_kernel<double>, grid_for(n16), dim3(kBlock), 0, st, n16, x, ar, ai, y);
    else hipLaunchKernelGGL(xpay_kernel<float>, grid_for(n16), dim3(kBlock), 0, st, n16, x, ar, ai, y);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblk, int ncol, double *sums, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, st, partials, nblk, ncol, sums);
    return hipGetLastError();
}

hipError_t launch_cg_alpha(const double *partials, int nblk, double *sc, hipStream_t st, double *hist)
{
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(kFinThreads), 0, st, partials, nblk, sc, hist);
    return hipGetLastError();
}

hipError_t launch_cg_beta(const double *partials, int nblk, double *sc, hipStream_t st)
{
    hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kFinThreads), 0, st, partials, nblk, sc);
    return hipGetLastError();
}

hipError_t launch_cg_update_r(int prec, size_t n16, void *r, const void *Ap, const double *sc, double *partials,
                              hipStream_t st)
{
    if (prec == HRD_F64) hipLaunchKernelGGL(cg_update_r_kernel<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, r, Ap, sc, partials);
    else hipLaunchKernelGGL(cg_update_r_kernel<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, r, Ap, sc, partials);
    return hipGetLastError();
}

hipError_t launch_cg_update_xp64(size_t n16, void *x, void *p, const void *r, const double *sc, hipStream_t st)
{
    hipLaunchKernelGGL(cg_update_xp64_kernel, grid_for(n16), dim3(kBlock), 0, st, n16, x, p, r, sc);
    return hipGetLastError();
}

hipError_t launch_cg_update_p32(size_t n16, void *p32, const void *r32, const double *sc, hipStream_t st)
{
    hipLaunchKernelGGL(cg_update_p32_kernel, grid_for(n16), dim3(kBlock), 0, st, n16, p32, r32, sc);
    return hipGetLastError();
}

hipError_t launch_cg_residual_mixed(int Vh, int ncomp, const void *b, const void *Ax, void *r64, void *r32,
                                    double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(cg_residual_mixed_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, st, Vh, ncomp / 2, b, Ax, r64, r32, partials);
    return hipGetLastError();
}

hipError_t launch_cg_residual64(size_t n16, const void *b, const void *Ax, void *r, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(cg_residual64_kernel, dim3(kRedBlocks), dim3(kRedThreads), 0, st, n16, b, Ax, r, partials);
    return hipGetLastError();
}

hipError_t launch_copy(size_t bytes, const void *src, void *dst, hipStream_t st)
{
    const size_t n = bytes / 16;
    if (n) hipLaunchKernelGGL(copy16_kernel, grid_for(n), dim3(kBlock), 0, st, n, (const float4 *)src, (float4 *)dst);
    return hipGetLastError();
}

hipError_t launch_zero(size_t bytes, void *dst, hipStream_t st)
{
    const size_t n = bytes / 16;
    if (n) hipLaunchKernelGGL(zero16_kernel, grid_for(n), dim3(kBlock), 0, st, n, (float4 *)dst);
    return hipGetLastError();
}

namespace {

// The ring of the mixed CG with p in F16 storage: one thread per site (the
// F16 site scale covers all components of the site); MODE bits as for
// cg_ring_f32_kernel.
template <int NC, int MODE>
__global__ __launch_bounds__(kBlock) void cg_ring_h16_kernel(int Vh, void *x64, char *ring, size_t stride, int m,
                                                             int src, int dst, const void *r32, const double *sc,
                                                             const double *ahist, int beta_mode)
{
    const int site = blockIdx.x * kBlock + threadIdx.x;
    if (site >= Vh) return;
    if constexpr ((MODE & 1) != 0) {
        Cx<double> x[NC];
        SpinorIO<double>::load<NC>(x64, Vh, site, x);
#pragma unroll 1
        for (int s = 0; s < m; s++) {
            const double alpha = ahist[s];
            Cx<float> p[NC];
            SpinorIO<h16>::load<NC>(ring + (size_t)s * stride, Vh, site, p);
#pragma unroll
            for (int k = 0; k < NC; k++) {
                x[k].re += alpha * (double)p[k].re;
                x[k].im += alpha * (double)p[k].im;
            }
        }
        SpinorIO<double>::store<NC>(x64, Vh, site, x);
    }
    if constexpr ((MODE & 2) != 0) {
        const float beta = ring_beta(sc, beta_mode);
        Cx<float> p[NC], r[NC];
        SpinorIO<h16>::load<NC>(ring + (size_t)src * stride, Vh, site, p);
        SpinorIO<float>::load<NC>(r32, Vh, site, r);
#pragma unroll
        for (int k = 0; k < NC; k++) p[k] = Cx<float>{r[k].re + beta * p[k].re, r[k].im + beta * p[k].im};
        SpinorIO<h16>::store<NC>(ring + (size_t)dst * stride, Vh, site, p);
    }
}

template <int MODE>
void launch_ring_h16(int Vh, int ncomp, void *x64, char *ring, size_t stride, int m, int src, int dst,
                     const void *r32, const double *sc, const double *ahist, int beta_mode, hipStream_t st)
{
    const dim3 grid((unsigned)((Vh + kBlock - 1) / kBlock));
#define HRD_RING16(NC) \
    hipLaunchKernelGGL((cg_ring_h16_kernel<NC, MODE>), grid, dim3(kBlock), 0, st, Vh, x64, ring, stride, m, src, dst, r32, sc, ahist, beta_mode)
    switch (ncomp) {
        case 8: HRD_RING16(8); break;
        case 12: HRD_RING16(12); break;
        case 16: HRD_RING16(16); break;
        case 24: HRD_RING16(24); break;
        case 32: HRD_RING16(32); break;
        case 40: HRD_RING16(40); break;
        default: HRD_RING16(60); break;
    }
#undef HRD_RING16
}

template <int MODE>
void launch_ring_f32(int Vh, int ncomp, void *x64, char *ring, size_t stride, int m, int src, int dst,
                     const void *r32, const double *sc, const double *ahist, int beta_mode, hipStream_t st)
{
    const int npl = ncomp / 2;
    hipLaunchKernelGGL((cg_ring_f32_kernel<MODE>), grid_for((size_t)npl * Vh), dim3(kBlock), 0, st, Vh, npl, x64,
                       ring, stride, m, src, dst, r32, sc, ahist, beta_mode);
}

}  // namespace

hipError_t launch_cg_ring(int prec, int Vh, int ncomp, void *x64, void *ring, size_t stride, int m, int src,
                          int dst, const void *r32, const double *sc, const double *ahist, int beta_mode, hipStream_t st)
{
    if (m < 0 || m > kPRing || (m == 0 && dst < 0)) return hipErrorInvalidValue;
    char *rg = static_cast<char *>(ring);
    const bool fl = m > 0, adv = dst >= 0;
    if (prec == HRD_F16) {
        if (fl && adv) launch_ring_h16<3>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
        else if (fl) launch_ring_h16<1>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
        else launch_ring_h16<2>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
    } else {
        if (fl && adv) launch_ring_f32<3>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
        else if (fl) launch_ring_f32<1>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
        else launch_ring_f32<2>(Vh, ncomp, x64, rg, stride, m, src, dst, r32, sc, ahist, beta_mode, st);
    }
    return hipGetLastError();
}

}  // namespace hrd
