// Device-side building blocks shared by the libhrd kernels: lattice geometry
// with even/odd site order, packed field layouts, complex arithmetic and
// deterministic block reductions.  Conventions are those stated in hrd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hrd.h"

namespace hrd {

constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels
constexpr int kNumXcd = 8;   // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kNumCu = 256;

// ---------------------------------------------------------------------------
// Unsigned division by a runtime constant via a 64-bit multiply: for
// n < 2^31 and S = 32 + ceil(log2 d), M = ceil(2^S / d) gives
// floor(n / d) = (n * M) >> S exactly (error term M d - 2^S < d <= 2^(S-32)).
// ---------------------------------------------------------------------------
struct FastDiv {
    uint64_t mul;
    uint32_t shift;
    uint32_t d;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t p = 0;
    while ((1u << p) < d) ++p;
    FastDiv f;
    f.shift = 32 + p;
    // ceil(2^S / d) computed without overflow: S <= 63 for d <= 2^31
    unsigned __int128 num = (unsigned __int128)1 << f.shift;
    f.mul = (uint64_t)((num + d - 1) / d);
    f.d = d;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return (uint32_t)(((uint64_t)n * f.mul) >> f.shift);
}

// ---------------------------------------------------------------------------
// Lattice geometry.  lex(x) = ((t L1 + x1) L2 + x2) L3 + x3; a site of
// parity p has index lex >> 1 in the parity-p block.
// ---------------------------------------------------------------------------
struct Geom {
    int L[4];       // {T, L1, L2, L3}
    int stride[4];  // lex strides {L1 L2 L3, L2 L3, L3, 1}
    int Vh;         // sites per parity
    FastDiv div3, div2, div1;
};

inline Geom make_geom(const int dims[4])
{
    Geom g;
    for (int i = 0; i < 4; i++) g.L[i] = dims[i];
    g.stride[3] = 1;
    g.stride[2] = dims[3];
    g.stride[1] = dims[3] * dims[2];
    g.stride[0] = dims[3] * dims[2] * dims[1];
    g.Vh = (int)((long long)dims[0] * dims[1] * dims[2] * dims[3] / 2);
    g.div3 = make_fastdiv(dims[3]);
    g.div2 = make_fastdiv(dims[2]);
    g.div1 = make_fastdiv(dims[1]);
    return g;
}

struct Site {
    int x[4];
    int lex;
};

// Coordinates of the site with index idx in the parity-p block.
__device__ __forceinline__ Site eo_site(const Geom &g, int idx, int p)
{
    Site s;
    const uint32_t c = 2u * (uint32_t)idx;  // lex of the even-x3 member of the pair
    const uint32_t q3 = fdiv(c, g.div3);
    const int x3e = (int)(c - q3 * (uint32_t)g.L[3]);
    const uint32_t q2 = fdiv(q3, g.div2);
    s.x[2] = (int)(q3 - q2 * (uint32_t)g.L[2]);
    const uint32_t q1 = fdiv(q2, g.div1);
    s.x[1] = (int)(q2 - q1 * (uint32_t)g.L[1]);
    s.x[0] = (int)q1;
    const int odd = (s.x[0] + s.x[1] + s.x[2] + p) & 1;
    s.x[3] = x3e + odd;
    s.lex = (int)c + odd;
    return s;
}

// eo index of the forward / backward neighbour in direction mu.
__device__ __forceinline__ int nbr_fwd(const Geom &g, const Site &s, int mu)
{
    const int l = (s.x[mu] == g.L[mu] - 1) ? s.lex - (g.L[mu] - 1) * g.stride[mu]
                                            : s.lex + g.stride[mu];
    return l >> 1;
}

__device__ __forceinline__ int nbr_bwd(const Geom &g, const Site &s, int mu)
{
    const int l = (s.x[mu] == 0) ? s.lex + (g.L[mu] - 1) * g.stride[mu]
                                 : s.lex - g.stride[mu];
    return l >> 1;
}

// ---------------------------------------------------------------------------
// XCD-aware block order: the hardware hands consecutive workgroups to the 8
// XCDs round-robin; remapping makes each XCD walk one contiguous range of the
// logical grid, so neighbouring sites share that XCD's L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_logical_block(int b, int nb)
{
    const int xcd = b % kNumXcd;
    const int slot = b / kNumXcd;
    const int q = nb / kNumXcd;
    const int r = nb % kNumXcd;
    return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// ---------------------------------------------------------------------------
// Complex numbers
// ---------------------------------------------------------------------------
template <typename R>
struct Cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ Cx<R> cx(R a, R b) { return Cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
// a * b
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc)
{
    return {acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re};
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cfmac(Cx<R> a, Cx<R> b, Cx<R> acc)
{
    return {acc.re + a.re * b.re + a.im * b.im, acc.im + a.re * b.im - a.im * b.re};
}
// i * a
template <typename R>
__device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return {-a.im, a.re}; }

// ---------------------------------------------------------------------------
// Packed spinor planes: F64 one complex128 per 16-byte element, F32 two
// complex64 per 16-byte element (components 2k, 2k+1 in plane k).
// ---------------------------------------------------------------------------
template <typename R>
struct SpinorIO;

template <>
struct SpinorIO<double> {
    template <int NC>
    __device__ __forceinline__ static void load(const void *base, int Vh, int site, Cx<double> (&c)[NC])
    {
        const double2 *p = reinterpret_cast<const double2 *>(base);
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const double2 v = p[(size_t)k * Vh + site];
            c[k] = Cx<double>{v.x, v.y};
        }
    }
    template <int NC>
    __device__ __forceinline__ static void store(void *base, int Vh, int site, const Cx<double> (&c)[NC])
    {
        double2 *p = reinterpret_cast<double2 *>(base);
#pragma unroll
        for (int k = 0; k < NC; k++) p[(size_t)k * Vh + site] = make_double2(c[k].re, c[k].im);
    }
};

template <>
struct SpinorIO<float> {
    template <int NC>
    __device__ __forceinline__ static void load(const void *base, int Vh, int site, Cx<float> (&c)[NC])
    {
        const float4 *p = reinterpret_cast<const float4 *>(base);
#pragma unroll
        for (int k = 0; k < NC / 2; k++) {
            const float4 v = p[(size_t)k * Vh + site];
            c[2 * k] = Cx<float>{v.x, v.y};
            c[2 * k + 1] = Cx<float>{v.z, v.w};
        }
    }
    template <int NC>
    __device__ __forceinline__ static void store(void *base, int Vh, int site, const Cx<float> (&c)[NC])
    {
        float4 *p = reinterpret_cast<float4 *>(base);
#pragma unroll
        for (int k = 0; k < NC / 2; k++)
            p[(size_t)k * Vh + site] = make_float4(c[2 * k].re, c[2 * k].im, c[2 * k + 1].re, c[2 * k + 1].im);
    }
};

// ---------------------------------------------------------------------------
// Packed links.  Block (parity p, direction mu) starts at byte
// (4 p + mu) * Vh * bytes_per_link.
// ---------------------------------------------------------------------------
template <int REP, typename R>
struct LinkIO;

template <typename R>
struct FundLink {
    Cx<R> u[2][2];
};
template <typename R>
struct AdjLink {
    R r[3][3];
};

__host__ __device__ constexpr int link_bytes(int rep, int prec)
{
    return rep == HRD_FUND ? (prec == HRD_F64 ? 64 : 32) : (prec == HRD_F64 ? 72 : 36);
}

__host__ __device__ constexpr int spinor_site_bytes(int rep, int prec)
{
    return (rep == HRD_FUND ? 8 : 12) * (prec == HRD_F64 ? 16 : 8);
}

template <>
struct LinkIO<HRD_FUND, double> {
    using Link = FundLink<double>;
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const double2 *b = reinterpret_cast<const double2 *>(U) + (size_t)(4 * p + mu) * Vh * 4;
        Link l;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const double2 v = b[(size_t)e * Vh + site];
            l.u[e >> 1][e & 1] = Cx<double>{v.x, v.y};
        }
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        double2 *b = reinterpret_cast<double2 *>(U) + (size_t)(4 * p + mu) * Vh * 4;
#pragma unroll
        for (int e = 0; e < 4; e++)
            b[(size_t)e * Vh + site] = make_double2(l.u[e >> 1][e & 1].re, l.u[e >> 1][e & 1].im);
    }
};

template <>
struct LinkIO<HRD_FUND, float> {
    using Link = FundLink<float>;
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const float4 *b = reinterpret_cast<const float4 *>(U) + (size_t)(4 * p + mu) * Vh * 2;
        Link l;
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const float4 v = b[(size_t)r * Vh + site];
            l.u[r][0] = Cx<float>{v.x, v.y};
            l.u[r][1] = Cx<float>{v.z, v.w};
        }
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        float4 *b = reinterpret_cast<float4 *>(U) + (size_t)(4 * p + mu) * Vh * 2;
#pragma unroll
        for (int r = 0; r < 2; r++)
            b[(size_t)r * Vh + site] = make_float4(l.u[r][0].re, l.u[r][0].im, l.u[r][1].re, l.u[r][1].im);
    }
};

template <>
struct LinkIO<HRD_ADJ, double> {
    using Link = AdjLink<double>;
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *blk = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 72;
        const double2 *b2 = reinterpret_cast<const double2 *>(blk);
        const double *b1 = reinterpret_cast<const double *>(blk + (size_t)Vh * 64);
        double e[9];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double2 v = b2[(size_t)k * Vh + site];
            e[2 * k] = v.x;
            e[2 * k + 1] = v.y;
        }
        e[8] = b1[site];
        Link l;
#pragma unroll
        for (int k = 0; k < 9; k++) l.r[k / 3][k % 3] = e[k];
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *blk = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 72;
        double2 *b2 = reinterpret_cast<double2 *>(blk);
        double *b1 = reinterpret_cast<double *>(blk + (size_t)Vh * 64);
#pragma unroll
        for (int k = 0; k < 4; k++)
            b2[(size_t)k * Vh + site] = make_double2(l.r[(2 * k) / 3][(2 * k) % 3], l.r[(2 * k + 1) / 3][(2 * k + 1) % 3]);
        b1[site] = l.r[2][2];
    }
};

template <>
struct LinkIO<HRD_ADJ, float> {
    using Link = AdjLink<float>;
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *blk = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 36;
        const float4 *b4 = reinterpret_cast<const float4 *>(blk);
        const float *b1 = reinterpret_cast<const float *>(blk + (size_t)Vh * 32);
        float e[9];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const float4 v = b4[(size_t)k * Vh + site];
            e[4 * k] = v.x;
            e[4 * k + 1] = v.y;
            e[4 * k + 2] = v.z;
            e[4 * k + 3] = v.w;
        }
        e[8] = b1[site];
        Link l;
#pragma unroll
        for (int k = 0; k < 9; k++) l.r[k / 3][k % 3] = e[k];
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *blk = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 36;
        float4 *b4 = reinterpret_cast<float4 *>(blk);
        float *b1 = reinterpret_cast<float *>(blk + (size_t)Vh * 32);
        float e[9];
#pragma unroll
        for (int k = 0; k < 9; k++) e[k] = l.r[k / 3][k % 3];
#pragma unroll
        for (int k = 0; k < 2; k++)
            b4[(size_t)k * Vh + site] = make_float4(e[4 * k], e[4 * k + 1], e[4 * k + 2], e[4 * k + 3]);
        b1[site] = e[8];
    }
};

// Colour multiplication of one spin component: out = U h, or U^+ h.
template <typename R>
__device__ __forceinline__ void link_mul(const FundLink<R> &l, const Cx<R> (&h)[2], Cx<R> (&o)[2])
{
    o[0] = cfma(l.u[0][1], h[1], cmul(l.u[0][0], h[0]));
    o[1] = cfma(l.u[1][1], h[1], cmul(l.u[1][0], h[0]));
}
template <typename R>
__device__ __forceinline__ void link_mul_dag(const FundLink<R> &l, const Cx<R> (&h)[2], Cx<R> (&o)[2])
{
    o[0] = cfmac(l.u[1][0], h[1], cmulc(l.u[0][0], h[0]));
    o[1] = cfmac(l.u[1][1], h[1], cmulc(l.u[0][1], h[0]));
}
template <typename R>
__device__ __forceinline__ void link_mul(const AdjLink<R> &l, const Cx<R> (&h)[3], Cx<R> (&o)[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
        o[i] = Cx<R>{l.r[i][0] * h[0].re + l.r[i][1] * h[1].re + l.r[i][2] * h[2].re,
                     l.r[i][0] * h[0].im + l.r[i][1] * h[1].im + l.r[i][2] * h[2].im};
}
template <typename R>
__device__ __forceinline__ void link_mul_dag(const AdjLink<R> &l, const Cx<R> (&h)[3], Cx<R> (&o)[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
        o[i] = Cx<R>{l.r[0][i] * h[0].re + l.r[1][i] * h[1].re + l.r[2][i] * h[2].re,
                     l.r[0][i] * h[0].im + l.r[1][i] * h[1].im + l.r[2][i] * h[2].im};
}

// ---------------------------------------------------------------------------
// Deterministic block sum of a double (wave64 butterfly, then LDS across the
// block's waves).  The result is valid in thread 0.  All threads must call.
// ---------------------------------------------------------------------------
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v)
{
    static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "block size");
    __shared__ double part[BLOCK / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; w++) s += part[w];
    }
    __syncthreads();
    return s;
}

template <int BLOCK>
__device__ __forceinline__ void block_sum2(double &a, double &b)
{
    static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "block size");
    __shared__ double part[2][BLOCK / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wave] = a;
        part[1][wave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; w++) {
            s0 += part[0][w];
            s1 += part[1][w];
        }
        a = s0;
        b = s1;
    }
    __syncthreads();
}

}  // namespace hrd
