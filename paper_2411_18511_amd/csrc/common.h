// Device-side building blocks shared by the libhrd kernels: lattice geometry
// with even/odd site order, packed field layouts, complex arithmetic and
// deterministic block reductions.  Conventions are those stated in hrd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

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
    int R;          // sites per parity in one (t, x1) row: L2 L3 / 2
    int B;          // x1-slab width of the traversal (divides L1)
    FastDiv div3, div2, div1;
    FastDiv divR, divB, divT;
};

// Slab width for the traversal of the hopping kernels: the lattice is swept
// in t inside x1-slabs of width B, so the t-neighbour rows of a sweep are
// B rows apart and stay in the XCD's L2.  B = L1 is plain lexicographic order.
int choose_slab(const int dims[4]);
// Slab width of the one-launch plain operator (both parities), per precision.
int choose_slab_full(const int dims[4], int prec);

inline Geom make_geom(const int dims[4], int slab = 0)
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
    g.R = dims[2] * dims[3] / 2;
    g.B = (slab > 0 && dims[1] % slab == 0) ? slab : choose_slab(dims);
    g.divR = make_fastdiv(g.R);
    g.divB = make_fastdiv(g.B);
    g.divT = make_fastdiv(dims[0]);
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

// Site of traversal position w (0 <= w < Vh) in the parity-p block, in slab
// order: w = ((s T + t) B + x1_in) R + k with x1 = s B + x1_in and k the
// position inside the (t, x1) row.  Rows are contiguous in the eo index, so
// consecutive w stay coalesced; *idx receives the eo index.
__device__ __forceinline__ Site slab_site(const Geom &g, int w, int p, int *idx)
{
    Site s;
    const uint32_t rr = fdiv((uint32_t)w, g.divR);
    const int k = w - (int)rr * g.R;
    const uint32_t q = fdiv(rr, g.divB);
    const int x1_in = (int)(rr - q * (uint32_t)g.B);
    const uint32_t sl = fdiv(q, g.divT);
    s.x[0] = (int)(q - sl * (uint32_t)g.L[0]);
    s.x[1] = (int)sl * g.B + x1_in;
    const uint32_t c = 2u * (uint32_t)k;
    const uint32_t x2 = fdiv(c, g.div3);
    s.x[2] = (int)x2;
    const int x3e = (int)(c - x2 * (uint32_t)g.L[3]);
    const int odd = (s.x[0] + s.x[1] + s.x[2] + p) & 1;
    s.x[3] = x3e + odd;
    const int row = s.x[0] * g.L[1] + s.x[1];
    *idx = row * g.R + k;
    s.lex = 2 * (*idx) + odd;
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
// 16-byte loads and stores, optionally non-temporal (streamed data that is
// used once: links in a hop, outputs)
// ---------------------------------------------------------------------------
typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ vd2 ld16d(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vd2 *>(p));
    else return *reinterpret_cast<const vd2 *>(p);
}
// The same load through a buffer resource based at `base`, with a 32-bit
// byte offset (the caller guarantees off < 2^31): the address of each load is
// one offset register added to a wave-uniform base instead of a 64-bit
// per-lane address, which measurably shortens the FP64 hopping kernel.
template <bool NT>
__device__ __forceinline__ vd2 ld16d_rel(const char *base, size_t off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(base), (short)0, 0x7fffffff, 0x00020000);
    return __builtin_bit_cast(vd2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, NT ? 2 : 0));
}
template <bool REL, bool NT>
__device__ __forceinline__ vd2 ld16d_at(const char *base, size_t off)
{
    if constexpr (REL) return ld16d_rel<NT>(base, off);
    else return ld16d<NT>(base + off);
}
template <bool NT>
__device__ __forceinline__ vf4 ld16f(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(p));
    else return *reinterpret_cast<const vf4 *>(p);
}
template <bool NT>
__device__ __forceinline__ void st16d(void *p, vd2 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vd2 *>(p));
    else *reinterpret_cast<vd2 *>(p) = v;
}
template <bool NT>
__device__ __forceinline__ void st16f(void *p, vf4 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vf4 *>(p));
    else *reinterpret_cast<vf4 *>(p) = v;
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
// Fused multiply-add with one rounding; with -ffp-contract=off these are the
// only fused operations, so a given expression rounds identically in every
// kernel that evaluates it.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a * b
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b)
{
    return {fmadd(a.re, b.re, -a.im * b.im), fmadd(a.re, b.im, a.im * b.re)};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b)
{
    return {fmadd(a.re, b.re, a.im * b.im), fmadd(a.re, b.im, -a.im * b.re)};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc)
{
    return {fmadd(a.re, b.re, fmadd(-a.im, b.im, acc.re)), fmadd(a.re, b.im, fmadd(a.im, b.re, acc.im))};
}
// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ Cx<R> cfmac(Cx<R> a, Cx<R> b, Cx<R> acc)
{
    return {fmadd(a.re, b.re, fmadd(a.im, b.im, acc.re)), fmadd(a.re, b.im, fmadd(-a.im, b.re, acc.im))};
}
// i * a
template <typename R>
__device__ __forceinline__ Cx<R> mul_i(Cx<R> a) { return {-a.im, a.re}; }

// ---------------------------------------------------------------------------
// Storage types.  A field's storage type S is double (F64), float (F32) or h16
// (F16: binary16 values); arithmetic runs in Arith<S>::type (FP32 for h16).
// ---------------------------------------------------------------------------
struct h16 {};
template <typename S>
struct Arith {
    using type = S;
};
template <>
struct Arith<h16> {
    using type = float;
};

typedef _Float16 vh8 __attribute__((ext_vector_type(8)));
typedef _Float16 vh4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ vh8 ld16h(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vh8 *>(p));
    else return *reinterpret_cast<const vh8 *>(p);
}
template <bool NT>
__device__ __forceinline__ void st16h(void *p, vh8 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vh8 *>(p));
    else *reinterpret_cast<vh8 *>(p) = v;
}
template <bool NT>
__device__ __forceinline__ vh4 ld8h(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vh4 *>(p));
    else return *reinterpret_cast<const vh4 *>(p);
}
template <typename T>
__device__ __forceinline__ T ld_scalar(const T *p, bool nt)
{
    return nt ? __builtin_nontemporal_load(p) : *p;
}
// binary16 of the FP32 rounding of x (round to nearest even at both steps)
template <typename T>
__device__ __forceinline__ _Float16 to_h16(T x) { return (_Float16)(float)x; }

// ---------------------------------------------------------------------------
// Packed spinor planes: F64 one complex128 per 16-byte element, F32 two
// complex64 per 16-byte element (components 2k, 2k+1 in plane k).
// ---------------------------------------------------------------------------
// 64-site tiles (spinor fields, FUND and ADJ links, FP64 first-row SU(2) links): a block of Vh sites (one
// parity of a spinor, one (parity, direction) of a gauge field) is a sequence
// of tiles; tile t holds, for its nb sites (64, the last tile the remaining
// ones), plane 0, then plane 1, ... (16-byte elements), and for F16 spinors
// then the nb FP32 site scales (ADJ links: the nb last entries).  A wave's loads of all planes of its sites
// thus fall into one contiguous stretch instead of one stream per plane.
// Byte offset of plane q of `site` in a block of P 16-byte planes and
// `extra` further bytes per site stored after the planes.
__host__ __device__ __forceinline__ size_t tile_off(int Vh, int site, int q, int P, int extra = 0)
{
    const int b0 = site & ~63;
    const int nb = Vh - b0 < 64 ? Vh - b0 : 64;
    return (size_t)b0 * (16 * P + extra) + ((size_t)q * nb + (size_t)(site - b0)) * 16;
}

// Byte offset of the trailing E-byte element of `site` (after P planes of 16
// bytes per site): the F16 spinor scale (E = 4), the last ADJ link entry.
__host__ __device__ __forceinline__ size_t tile_extra_off(int Vh, int site, int P, int E)
{
    const int b0 = site & ~63;
    const int nb = Vh - b0 < 64 ? Vh - b0 : 64;
    return (size_t)b0 * (16 * P + E) + (size_t)P * nb * 16 + (size_t)(site - b0) * E;
}
__host__ __device__ __forceinline__ size_t tile_scale_off(int Vh, int site, int P)
{
    return tile_extra_off(Vh, site, P, 4);
}

// Fields that pair an FP32 spinor (npl planes, components 2q, 2q+1 in plane
// q) with an FP64 one (2 npl planes): for an index t over (F32 plane q, site
// j), q slow, the byte offsets of F32 plane q and of F64 planes 2q, 2q+1.
struct MixOff {
    size_t f32, f64a, f64b;
};
__device__ __forceinline__ MixOff mix_off(long t, int Vh, int npl)
{
    const int q = (int)(t / Vh);
    const int j = (int)(t - (long)q * Vh);
    return MixOff{tile_off(Vh, j, q, npl), tile_off(Vh, j, 2 * q, 2 * npl), tile_off(Vh, j, 2 * q + 1, 2 * npl)};
}

template <typename R>
struct SpinorIO;

template <>
struct SpinorIO<double> {
    // REL: 32-bit offsets from the block base (the block is below 2 GiB)
    template <int NC, bool NT = false, bool REL = false>
    __device__ __forceinline__ static void load(const void *base, int Vh, int site, Cx<double> (&c)[NC])
    {
        const char *p = reinterpret_cast<const char *>(base);
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const vd2 v = ld16d_at<REL, NT>(p, tile_off(Vh, site, k, NC));
            c[k] = Cx<double>{v.x, v.y};
        }
    }
    template <int NC, bool NT = false>
    __device__ __forceinline__ static void store(void *base, int Vh, int site, const Cx<double> (&c)[NC])
    {
        char *p = reinterpret_cast<char *>(base);
#pragma unroll
        for (int k = 0; k < NC; k++) st16d<NT>(p + tile_off(Vh, site, k, NC), vd2{c[k].re, c[k].im});
    }
};

template <>
struct SpinorIO<float> {
    template <int NC, bool NT = false, bool REL = false>
    __device__ __forceinline__ static void load(const void *base, int Vh, int site, Cx<float> (&c)[NC])
    {
        const char *p = reinterpret_cast<const char *>(base);
#pragma unroll
        for (int k = 0; k < NC / 2; k++) {
            const vf4 v = ld16f<NT>(p + tile_off(Vh, site, k, NC / 2));
            c[2 * k] = Cx<float>{v.x, v.y};
            c[2 * k + 1] = Cx<float>{v.z, v.w};
        }
    }
    template <int NC, bool NT = false>
    __device__ __forceinline__ static void store(void *base, int Vh, int site, const Cx<float> (&c)[NC])
    {
        char *p = reinterpret_cast<char *>(base);
#pragma unroll
        for (int k = 0; k < NC / 2; k++)
            st16f<NT>(p + tile_off(Vh, site, k, NC / 2),
                      vf4{c[2 * k].re, c[2 * k].im, c[2 * k + 1].re, c[2 * k + 1].im});
    }
};

// F16: NC/4 planes of 16-byte elements, each holding four components as eight
// binary16 (re, im, re, im, ...) divided by the site scale s, followed in each
// tile by the FP32 s of its sites (4 bytes per site).  s is the largest |re| or |im| of the
// site; the stored values are binary16(x * (1/s)) with FP32 x, and a site with
// s = 0 stores zeros.  Reading gives binary16 * s in FP32.
template <>
struct SpinorIO<h16> {
    template <int NC, bool NT = false, bool REL = false>
    __device__ __forceinline__ static void load(const void *base, int Vh, int site, Cx<float> (&c)[NC])
    {
        // plane 0 of the site and the distance between planes, computed once;
        // all planes and the scale are loaded before any is converted
        constexpr int P = NC / 4;
        const int b0 = site & ~63, off = site - b0;
        const size_t step = (size_t)(Vh - b0 < 64 ? Vh - b0 : 64) * 16;  // nb 16-byte elements
        const char *tile = reinterpret_cast<const char *>(base) + (size_t)b0 * (16 * P + 4);
        const char *p0 = tile + (size_t)off * 16;
        vh8 v[P];
#pragma unroll
        for (int k = 0; k < P; k++) v[k] = ld16h<NT>(p0 + k * step);
        const float s = ld_scalar(reinterpret_cast<const float *>(tile + P * step + (size_t)off * 4), NT);
#pragma unroll
        for (int k = 0; k < P; k++)
#pragma unroll
            for (int j = 0; j < 4; j++) c[4 * k + j] = Cx<float>{(float)v[k][2 * j] * s, (float)v[k][2 * j + 1] * s};
    }
    // the stored value exactly (binary16 * s in FP64), for conversions to F64
    template <int NC>
    __device__ __forceinline__ static void load_exact(const void *base, int Vh, int site, Cx<double> (&c)[NC])
    {
        const char *p = reinterpret_cast<const char *>(base);
        const double s = *reinterpret_cast<const float *>(p + tile_scale_off(Vh, site, NC / 4));
#pragma unroll
        for (int k = 0; k < NC / 4; k++) {
            const vh8 v = ld16h<false>(p + tile_off(Vh, site, k, NC / 4, 4));
#pragma unroll
            for (int j = 0; j < 4; j++) c[4 * k + j] = Cx<double>{(double)v[2 * j] * s, (double)v[2 * j + 1] * s};
        }
    }
    template <int NC, bool NT = false>
    __device__ __forceinline__ static void store(void *base, int Vh, int site, const Cx<float> (&c)[NC])
    {
        char *p = reinterpret_cast<char *>(base);
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < NC; k++) m = fmaxf(m, fmaxf(fabsf(c[k].re), fabsf(c[k].im)));
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
        for (int k = 0; k < NC / 4; k++) {
            vh8 v;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                v[2 * j] = (_Float16)(c[4 * k + j].re * inv);
                v[2 * j + 1] = (_Float16)(c[4 * k + j].im * inv);
            }
            st16h<NT>(p + tile_off(Vh, site, k, NC / 4, 4), v);
        }
        float *sp = reinterpret_cast<float *>(p + tile_scale_off(Vh, site, NC / 4));
        if constexpr (NT) __builtin_nontemporal_store(m, sp);
        else *sp = m;
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

__host__ __device__ constexpr bool is_su2_row(int rep) { return rep == HRD_FUND_SU2 || rep == HRD_ADJ_SU2; }

// Number of colours of the fermion in a representation.
__host__ __device__ constexpr int ncolour(int rep)
{
    return (rep == HRD_FUND || rep == HRD_FUND_SU2) ? 2
           : (rep == HRD_ADJ || rep == HRD_ADJ_SU2 || rep == HRD_CPLX3 || rep == HRD_SU3_ROW2) ? 3
           : rep == HRD_CPLX4 ? 4
           : rep == HRD_CPLX6 ? 6
           : rep == HRD_CPLX10 ? 10
           : rep == HRD_REAL15 ? 15
           : 8;
}

// Dense link formats of SU(N > 2) representations.
__host__ __device__ constexpr bool is_dense(int rep) { return rep >= HRD_CPLX3; }
__host__ __device__ constexpr bool is_real_dense(int rep) { return rep == HRD_REAL8 || rep == HRD_REAL15; }
// Formats the clover term supports: the SU(2) ones and SU(3) fundamental links.
__host__ __device__ constexpr bool clover_capable(int rep)
{
    return !is_dense(rep) || rep == HRD_CPLX3 || rep == HRD_SU3_ROW2;
}

// Representation whose (uncompressed) layout a derivative with respect to the
// links uses: FUND for FUND and FUND_SU2, ADJ for ADJ and ADJ_SU2, the format
// itself for the dense formats.
__host__ __device__ constexpr int base_rep(int rep)
{
    return rep == HRD_SU3_ROW2 ? HRD_CPLX3 : is_dense(rep) ? rep : ncolour(rep) == 2 ? HRD_FUND : HRD_ADJ;
}

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Bytes per link.  SU(2) formats: real entries (8 FUND, 9 ADJ, 4 for a first
// row) times the storage width (8 F64, 4 F32, 2 F16).  Dense formats: whole
// 16-byte planes, n^2 complex or real entries packed in order.
__host__ __device__ constexpr int link_bytes(int rep, int prec)
{
    return rep == HRD_SU3_ROW2 ? (prec == HRD_F64 ? 96 : prec == HRD_F32 ? 48 : 24)
           : is_dense(rep)
               ? 16 * ceil_div(ncolour(rep) * ncolour(rep),
                               (is_real_dense(rep) ? 2 : 1) * (prec == HRD_F64 ? 1 : prec == HRD_F32 ? 2 : 4))
               : (is_su2_row(rep) ? 4 : rep == HRD_FUND ? 8 : 9) * (prec == HRD_F64 ? 8 : prec == HRD_F32 ? 4 : 2);
}

// Bytes per site of a spinor: 4N complex components; F16 adds the FP32 site scale.
__host__ __device__ constexpr int spinor_site_bytes(int rep, int prec)
{
    return prec == HRD_F16 ? 4 * ncolour(rep) * 4 + 4 : 4 * ncolour(rep) * (prec == HRD_F64 ? 16 : 8);
}

template <>
struct LinkIO<HRD_FUND, double> {
    using Link = FundLink<double>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 64;
        Link l;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const vd2 v = ld16d_at<REL, NT>(b, tile_off(Vh, site, e, 4));
            l.u[e >> 1][e & 1] = Cx<double>{v.x, v.y};
        }
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 64;
#pragma unroll
        for (int e = 0; e < 4; e++)
            st16d<false>(b + tile_off(Vh, site, e, 4), vd2{l.u[e >> 1][e & 1].re, l.u[e >> 1][e & 1].im});
    }
};

template <>
struct LinkIO<HRD_FUND, float> {
    using Link = FundLink<float>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 32;
        Link l;
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const vf4 v = ld16f<NT>(b + tile_off(Vh, site, r, 2));
            l.u[r][0] = Cx<float>{v.x, v.y};
            l.u[r][1] = Cx<float>{v.z, v.w};
        }
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 32;
#pragma unroll
        for (int r = 0; r < 2; r++)
            st16f<false>(b + tile_off(Vh, site, r, 2), vf4{l.u[r][0].re, l.u[r][0].im, l.u[r][1].re, l.u[r][1].im});
    }
};

template <>
struct LinkIO<HRD_ADJ, double> {
    using Link = AdjLink<double>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *blk = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 72;
        const double *b1 = reinterpret_cast<const double *>(blk + tile_extra_off(Vh, site, 4, 8));
        double e[9];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const vd2 v = ld16d_at<REL, NT>(blk, tile_off(Vh, site, k, 4, 8));
            e[2 * k] = v.x;
            e[2 * k + 1] = v.y;
        }
        if constexpr (NT) e[8] = __builtin_nontemporal_load(b1);
        else e[8] = *b1;
        Link l;
#pragma unroll
        for (int k = 0; k < 9; k++) l.r[k / 3][k % 3] = e[k];
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *blk = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 72;
        double *b1 = reinterpret_cast<double *>(blk + tile_extra_off(Vh, site, 4, 8));
        double e[9];
#pragma unroll
        for (int k = 0; k < 9; k++) e[k] = l.r[k / 3][k % 3];
#pragma unroll
        for (int k = 0; k < 4; k++) st16d<false>(blk + tile_off(Vh, site, k, 4, 8), vd2{e[2 * k], e[2 * k + 1]});
        *b1 = e[8];
    }
};

template <>
struct LinkIO<HRD_ADJ, float> {
    using Link = AdjLink<float>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *blk = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 36;
        const float *b1 = reinterpret_cast<const float *>(blk + tile_extra_off(Vh, site, 2, 4));
        float e[9];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const vf4 v = ld16f<NT>(blk + tile_off(Vh, site, k, 2, 4));
            e[4 * k] = v.x;
            e[4 * k + 1] = v.y;
            e[4 * k + 2] = v.z;
            e[4 * k + 3] = v.w;
        }
        if constexpr (NT) e[8] = __builtin_nontemporal_load(b1);
        else e[8] = *b1;
        Link l;
#pragma unroll
        for (int k = 0; k < 9; k++) l.r[k / 3][k % 3] = e[k];
        return l;
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Link &l)
    {
        char *blk = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 36;
        float *b1 = reinterpret_cast<float *>(blk + tile_extra_off(Vh, site, 2, 4));
        float e[9];
#pragma unroll
        for (int k = 0; k < 9; k++) e[k] = l.r[k / 3][k % 3];
#pragma unroll
        for (int k = 0; k < 2; k++)
            st16f<false>(blk + tile_off(Vh, site, k, 2, 4), vf4{e[4 * k], e[4 * k + 1], e[4 * k + 2], e[4 * k + 3]});
        *b1 = e[8];
    }
};

// First row (a, b) of an SU(2) link U = [[a, b], [-conj(b), conj(a)]].
template <typename R>
struct Su2Row {
    Cx<R> a, b;
};

template <typename R>
struct RowIO;

template <>
struct RowIO<double> {
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Su2Row<double> load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 32;
        const vd2 x = ld16d_at<REL, NT>(b, tile_off(Vh, site, 0, 2));
        const vd2 y = ld16d_at<REL, NT>(b, tile_off(Vh, site, 1, 2));
        return Su2Row<double>{{x.x, x.y}, {y.x, y.y}};
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Su2Row<double> &r)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 32;
        st16d<false>(b + tile_off(Vh, site, 0, 2), vd2{r.a.re, r.a.im});
        st16d<false>(b + tile_off(Vh, site, 1, 2), vd2{r.b.re, r.b.im});
    }
};

template <>
struct RowIO<float> {
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Su2Row<float> load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 16;
        const vf4 v = ld16f<NT>(b + (size_t)site * 16);
        return Su2Row<float>{{v.x, v.y}, {v.z, v.w}};
    }
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Su2Row<float> &r)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 16;
        st16f<false>(b + (size_t)site * 16, vf4{r.a.re, r.a.im, r.b.re, r.b.im});
    }
};

// F16 links: binary16 entries, no scale (entries of unitary and orthogonal
// matrices are bounded by 1).  FUND: one 16-byte plane (U00, U01, U10, U11 as
// re, im).  ADJ: a 16-byte plane with entries 0-7 and a 2-byte plane with
// entry 8.  First row: one 8-byte plane (U00, U01).
template <>
struct LinkIO<HRD_FUND, h16> {
    using Link = FundLink<float>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 16;
        const vh8 v = ld16h<NT>(b + (size_t)site * 16);
        Link l;
#pragma unroll
        for (int e = 0; e < 4; e++) l.u[e >> 1][e & 1] = Cx<float>{(float)v[2 * e], (float)v[2 * e + 1]};
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const FundLink<T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 16;
        vh8 v;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            v[2 * e] = to_h16(l.u[e >> 1][e & 1].re);
            v[2 * e + 1] = to_h16(l.u[e >> 1][e & 1].im);
        }
        st16h<false>(b + (size_t)site * 16, v);
    }
};

template <>
struct LinkIO<HRD_ADJ, h16> {
    using Link = AdjLink<float>;
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *blk = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 18;
        const vh8 v = ld16h<NT>(blk + tile_off(Vh, site, 0, 1, 2));
        const _Float16 e8 = ld_scalar(reinterpret_cast<const _Float16 *>(blk + tile_extra_off(Vh, site, 1, 2)), NT);
        Link l;
#pragma unroll
        for (int k = 0; k < 8; k++) l.r[k / 3][k % 3] = (float)v[k];
        l.r[2][2] = (float)e8;
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const AdjLink<T> &l)
    {
        char *blk = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 18;
        vh8 v;
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = to_h16(l.r[k / 3][k % 3]);
        st16h<false>(blk + tile_off(Vh, site, 0, 1, 2), v);
        *reinterpret_cast<_Float16 *>(blk + tile_extra_off(Vh, site, 1, 2)) = to_h16(l.r[2][2]);
    }
};

template <>
struct RowIO<h16> {
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Su2Row<float> load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * 8;
        const vh4 v = ld8h<NT>(b + (size_t)site * 8);
        return Su2Row<float>{{(float)v[0], (float)v[1]}, {(float)v[2], (float)v[3]}};
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const Su2Row<T> &r)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * 8;
        vh4 v;
        v[0] = to_h16(r.a.re);
        v[1] = to_h16(r.a.im);
        v[2] = to_h16(r.b.re);
        v[3] = to_h16(r.b.im);
        *reinterpret_cast<vh4 *>(b + (size_t)site * 8) = v;
    }
};

template <typename R>
struct LinkIO<HRD_FUND_SU2, R> {
    using Link = FundLink<typename Arith<R>::type>;
    // second row reconstructed: U10 = -conj(U01), U11 = conj(U00)
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const auto r = RowIO<R>::template load<NT, REL>(U, Vh, p, mu, site);
        Link l;
        l.u[0][0] = r.a;
        l.u[0][1] = r.b;
        l.u[1][0] = {-r.b.re, r.b.im};
        l.u[1][1] = {r.a.re, -r.a.im};
        return l;
    }
};

template <typename R>
struct LinkIO<HRD_ADJ_SU2, R> {
    using A = typename Arith<R>::type;
    using Link = AdjLink<A>;
    // R(U)_ij = (a0^2 - |v|^2) d_ij + 2 v_i v_j + 2 a0 eps_ijk v_k for
    // U = a0 + i (v1 s1 + v2 s2 + v3 s3), read from the first row
    // a = a0 + i v3, b = v2 + i v1; this equals tr(s_i U s_j U^+) / 2 for
    // every U of that form (both sides are quadratic and agree on SU(2)).
    template <bool NT = false, bool REL = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const auto r = RowIO<R>::template load<NT, REL>(U, Vh, p, mu, site);
        const A a0 = r.a.re, v0 = r.b.im, v1 = r.b.re, v2 = r.a.im;
        const A d = a0 * a0 - (v0 * v0 + v1 * v1 + v2 * v2);
        const A t0 = 2 * a0 * v0, t1 = 2 * a0 * v1, t2 = 2 * a0 * v2;
        Link l;
        l.r[0][0] = d + 2 * v0 * v0;
        l.r[1][1] = d + 2 * v1 * v1;
        l.r[2][2] = d + 2 * v2 * v2;
        l.r[0][1] = 2 * v0 * v1 + t2;
        l.r[1][0] = 2 * v0 * v1 - t2;
        l.r[1][2] = 2 * v1 * v2 + t0;
        l.r[2][1] = 2 * v1 * v2 - t0;
        l.r[2][0] = 2 * v2 * v0 + t1;
        l.r[0][2] = 2 * v2 * v0 - t1;
        return l;
    }
};

// ---------------------------------------------------------------------------
// Dense links of SU(N > 2) representations: N x N complex (CPLXn) or real
// (REAL8), entries e = N i + j packed in order into 16-byte planes holding one
// complex128 / two complex64 / four binary16 complex (CPLXn), or two float64 /
// four float32 / eight binary16 (REAL8); the last plane is zero-padded.
// ---------------------------------------------------------------------------
template <int N, typename R>
struct CLink {
    Cx<R> u[N][N];
};
template <int N, typename R>
struct RLink {
    R r[N][N];
};

template <int N, typename S>
struct CplxIO;

template <int N>
struct CplxIO<N, double> {
    static constexpr int kPlanes = N * N;
    using Link = CLink<N, double>;
    // row I of the link (entries N I .. N I + N - 1)
    template <int I, bool NT = false>
    __device__ __forceinline__ static void load_row(const void *U, int Vh, int p, int mu, int site, Cx<double> (&row)[N])
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
#pragma unroll
        for (int j = 0; j < N; j++) {
            const vd2 v = ld16d<NT>(b + ((size_t)(N * I + j) * Vh + site) * 16);
            row[j] = Cx<double>{v.x, v.y};
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        Link l;
#pragma unroll
        for (int e = 0; e < N * N; e++) {
            const vd2 v = ld16d<NT>(b + ((size_t)e * Vh + site) * 16);
            l.u[e / N][e % N] = Cx<double>{v.x, v.y};
        }
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const CLink<N, T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
#pragma unroll
        for (int e = 0; e < N * N; e++)
            st16d<false>(b + ((size_t)e * Vh + site) * 16, vd2{(double)l.u[e / N][e % N].re, (double)l.u[e / N][e % N].im});
    }
};

template <int N>
struct CplxIO<N, float> {
    static constexpr int kPlanes = (N * N + 1) / 2;
    using Link = CLink<N, float>;
    template <int I, bool NT = false>
    __device__ __forceinline__ static void load_row(const void *U, int Vh, int p, int mu, int site, Cx<float> (&row)[N])
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        constexpr int e0 = N * I, e1 = N * I + N;
#pragma unroll
        for (int q = e0 / 2; q <= (e1 - 1) / 2; q++) {
            const vf4 v = ld16f<NT>(b + ((size_t)q * Vh + site) * 16);
            if (2 * q >= e0) row[2 * q - e0] = Cx<float>{v.x, v.y};
            if (2 * q + 1 < e1) row[2 * q + 1 - e0] = Cx<float>{v.z, v.w};
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        Link l;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            const vf4 v = ld16f<NT>(b + ((size_t)q * Vh + site) * 16);
            l.u[(2 * q) / N][(2 * q) % N] = Cx<float>{v.x, v.y};
            if (2 * q + 1 < N * N) l.u[(2 * q + 1) / N][(2 * q + 1) % N] = Cx<float>{v.z, v.w};
        }
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const CLink<N, T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            const int e0 = 2 * q, e1 = 2 * q + 1;
            const Cx<T> a = l.u[e0 / N][e0 % N];
            const Cx<T> c = e1 < N * N ? l.u[e1 / N][e1 % N] : Cx<T>{0, 0};
            st16f<false>(b + ((size_t)q * Vh + site) * 16, vf4{(float)a.re, (float)a.im, (float)c.re, (float)c.im});
        }
    }
};

template <int N>
struct CplxIO<N, h16> {
    static constexpr int kPlanes = (N * N + 3) / 4;
    using Link = CLink<N, float>;
    template <int I, bool NT = false>
    __device__ __forceinline__ static void load_row(const void *U, int Vh, int p, int mu, int site, Cx<float> (&row)[N])
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        constexpr int e0 = N * I, e1 = N * I + N;
#pragma unroll
        for (int q = e0 / 4; q <= (e1 - 1) / 4; q++) {
            const vh8 v = ld16h<NT>(b + ((size_t)q * Vh + site) * 16);
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (4 * q + j >= e0 && 4 * q + j < e1)
                    row[4 * q + j - e0] = Cx<float>{(float)v[2 * j], (float)v[2 * j + 1]};
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        Link l;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            const vh8 v = ld16h<NT>(b + ((size_t)q * Vh + site) * 16);
#pragma unroll
            for (int j = 0; j < 4; j++)
                if (4 * q + j < N * N)
                    l.u[(4 * q + j) / N][(4 * q + j) % N] = Cx<float>{(float)v[2 * j], (float)v[2 * j + 1]};
        }
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const CLink<N, T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            vh8 v;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int e = 4 * q + j;
                const Cx<T> a = e < N * N ? l.u[e / N][e % N] : Cx<T>{0, 0};
                v[2 * j] = to_h16(a.re);
                v[2 * j + 1] = to_h16(a.im);
            }
            st16h<false>(b + ((size_t)q * Vh + site) * 16, v);
        }
    }
};

template <int N, typename S>
struct RealIO {
    // reals per 16-byte plane: 2 (F64), 4 (F32), 8 (F16)
    static constexpr int kPer = std::is_same<S, double>::value ? 2 : std::is_same<S, float>::value ? 4 : 8;
    static constexpr int kPlanes = (N * N + kPer - 1) / kPer;
    using A = typename Arith<S>::type;
    using Link = RLink<N, A>;
    template <int I, bool NT = false>
    __device__ __forceinline__ static void load_row(const void *U, int Vh, int p, int mu, int site, A (&row)[N])
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        constexpr int e0 = N * I, e1 = N * I + N;
#pragma unroll
        for (int q = e0 / kPer; q <= (e1 - 1) / kPer; q++) {
            const char *a = b + ((size_t)q * Vh + site) * 16;
            A e[kPer];
            if constexpr (kPer == 2) {
                const vd2 v = ld16d<NT>(a);
                e[0] = v.x;
                e[1] = v.y;
            } else if constexpr (kPer == 4) {
                const vf4 v = ld16f<NT>(a);
                e[0] = v.x;
                e[1] = v.y;
                e[2] = v.z;
                e[3] = v.w;
            } else {
                const vh8 v = ld16h<NT>(a);
#pragma unroll
                for (int j = 0; j < 8; j++) e[j] = (float)v[j];
            }
#pragma unroll
            for (int j = 0; j < kPer; j++)
                if (kPer * q + j >= e0 && kPer * q + j < e1) row[kPer * q + j - e0] = e[j];
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
        Link l;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            const char *a = b + ((size_t)q * Vh + site) * 16;
            A e[kPer];
            if constexpr (kPer == 2) {
                const vd2 v = ld16d<NT>(a);
                e[0] = v.x;
                e[1] = v.y;
            } else if constexpr (kPer == 4) {
                const vf4 v = ld16f<NT>(a);
                e[0] = v.x;
                e[1] = v.y;
                e[2] = v.z;
                e[3] = v.w;
            } else {
                const vh8 v = ld16h<NT>(a);
#pragma unroll
                for (int j = 0; j < 8; j++) e[j] = (float)v[j];
            }
#pragma unroll
            for (int j = 0; j < kPer; j++)
                if (kPer * q + j < N * N) l.r[(kPer * q + j) / N][(kPer * q + j) % N] = e[j];
        }
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const RLink<N, T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * kPlanes * 16;
#pragma unroll
        for (int q = 0; q < kPlanes; q++) {
            char *a = b + ((size_t)q * Vh + site) * 16;
            T e[kPer];
#pragma unroll
            for (int j = 0; j < kPer; j++) {
                const int k = kPer * q + j;
                e[j] = k < N * N ? l.r[k / N][k % N] : T(0);
            }
            if constexpr (kPer == 2) {
                st16d<false>(a, vd2{(double)e[0], (double)e[1]});
            } else if constexpr (kPer == 4) {
                st16f<false>(a, vf4{(float)e[0], (float)e[1], (float)e[2], (float)e[3]});
            } else {
                vh8 v;
#pragma unroll
                for (int j = 0; j < 8; j++) v[j] = to_h16(e[j]);
                st16h<false>(a, v);
            }
        }
    }
};

// SU(3) links stored as their first two rows (6 complex entries, row-major);
// the third row is the complex conjugate of the cross product of the first
// two (exact for SU(3): det U = 1 and U unitary).  Planes: F64 six complex128,
// F32 three of 2 x complex64, F16 one 16-byte plane (entries 0-3) and one
// 8-byte plane (entries 4, 5).
template <typename S>
struct LinkIO<HRD_SU3_ROW2, S> {
    using A = typename Arith<S>::type;
    using Link = CLink<3, A>;
    static constexpr size_t kBytes = std::is_same<S, double>::value ? 96 : std::is_same<S, float>::value ? 48 : 24;
    template <bool NT = false>
    __device__ __forceinline__ static void load_rows01(const void *U, int Vh, int p, int mu, int site, Cx<A> (&e)[6])
    {
        const char *b = reinterpret_cast<const char *>(U) + (size_t)(4 * p + mu) * Vh * kBytes;
        if constexpr (std::is_same<S, double>::value) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const vd2 v = ld16d<NT>(b + ((size_t)k * Vh + site) * 16);
                e[k] = Cx<A>{v.x, v.y};
            }
        } else if constexpr (std::is_same<S, float>::value) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const vf4 v = ld16f<NT>(b + ((size_t)q * Vh + site) * 16);
                e[2 * q] = Cx<A>{v.x, v.y};
                e[2 * q + 1] = Cx<A>{v.z, v.w};
            }
        } else {
            const vh8 v = ld16h<NT>(b + (size_t)site * 16);
            const vh4 w = ld8h<NT>(b + (size_t)Vh * 16 + (size_t)site * 8);
#pragma unroll
            for (int k = 0; k < 4; k++) e[k] = Cx<A>{(float)v[2 * k], (float)v[2 * k + 1]};
            e[4] = Cx<A>{(float)w[0], (float)w[1]};
            e[5] = Cx<A>{(float)w[2], (float)w[3]};
        }
    }
    // row 2 = conj(row 0 x row 1)
    __device__ __forceinline__ static void third_row(const Cx<A> (&e)[6], Cx<A> (&r)[3])
    {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int i = (k + 1) % 3, j = (k + 2) % 3;
            const Cx<A> z = cmul(e[i], e[3 + j]) - cmul(e[j], e[3 + i]);
            r[k] = Cx<A>{z.re, -z.im};
        }
    }
    template <int I, bool NT = false>
    __device__ __forceinline__ static void load_row(const void *U, int Vh, int p, int mu, int site, Cx<A> (&row)[3])
    {
        Cx<A> e[6];
        load_rows01<NT>(U, Vh, p, mu, site, e);
        if constexpr (I < 2) {
#pragma unroll
            for (int k = 0; k < 3; k++) row[k] = e[3 * I + k];
        } else {
            third_row(e, row);
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static Link load(const void *U, int Vh, int p, int mu, int site)
    {
        Cx<A> e[6];
        load_rows01<NT>(U, Vh, p, mu, site, e);
        Link l;
#pragma unroll
        for (int k = 0; k < 6; k++) l.u[k / 3][k % 3] = e[k];
        Cx<A> r[3];
        third_row(e, r);
#pragma unroll
        for (int k = 0; k < 3; k++) l.u[2][k] = r[k];
        return l;
    }
    template <typename T>
    __device__ __forceinline__ static void store(void *U, int Vh, int p, int mu, int site, const CLink<3, T> &l)
    {
        char *b = reinterpret_cast<char *>(U) + (size_t)(4 * p + mu) * Vh * kBytes;
        Cx<T> e[6];
#pragma unroll
        for (int k = 0; k < 6; k++) e[k] = l.u[k / 3][k % 3];
        if constexpr (std::is_same<S, double>::value) {
#pragma unroll
            for (int k = 0; k < 6; k++) st16d<false>(b + ((size_t)k * Vh + site) * 16, vd2{(double)e[k].re, (double)e[k].im});
        } else if constexpr (std::is_same<S, float>::value) {
#pragma unroll
            for (int q = 0; q < 3; q++)
                st16f<false>(b + ((size_t)q * Vh + site) * 16, vf4{(float)e[2 * q].re, (float)e[2 * q].im,
                                                                    (float)e[2 * q + 1].re, (float)e[2 * q + 1].im});
        } else {
            vh8 v;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                v[2 * k] = to_h16(e[k].re);
                v[2 * k + 1] = to_h16(e[k].im);
            }
            st16h<false>(b + (size_t)site * 16, v);
            vh4 w;
            w[0] = to_h16(e[4].re);
            w[1] = to_h16(e[4].im);
            w[2] = to_h16(e[5].re);
            w[3] = to_h16(e[5].im);
            *reinterpret_cast<vh4 *>(b + (size_t)Vh * 16 + (size_t)site * 8) = w;
        }
    }
};

template <typename S>
struct LinkIO<HRD_CPLX3, S> : CplxIO<3, S> {};
template <typename S>
struct LinkIO<HRD_CPLX4, S> : CplxIO<4, S> {};
template <typename S>
struct LinkIO<HRD_CPLX6, S> : CplxIO<6, S> {};
template <typename S>
struct LinkIO<HRD_REAL8, S> : RealIO<8, S> {};
template <typename S>
struct LinkIO<HRD_CPLX10, S> : CplxIO<10, S> {};
template <typename S>
struct LinkIO<HRD_REAL15, S> : RealIO<15, S> {};

template <int N, typename R>
__device__ __forceinline__ void link_mul(const CLink<N, R> &l, const Cx<R> (&h)[N], Cx<R> (&o)[N])
{
#pragma unroll
    for (int i = 0; i < N; i++) {
        Cx<R> z = cmul(l.u[i][0], h[0]);
#pragma unroll
        for (int j = 1; j < N; j++) z = cfma(l.u[i][j], h[j], z);
        o[i] = z;
    }
}
template <int N, typename R>
__device__ __forceinline__ void link_mul_dag(const CLink<N, R> &l, const Cx<R> (&h)[N], Cx<R> (&o)[N])
{
#pragma unroll
    for (int i = 0; i < N; i++) {
        Cx<R> z = cmulc(l.u[0][i], h[0]);
#pragma unroll
        for (int j = 1; j < N; j++) z = cfmac(l.u[j][i], h[j], z);
        o[i] = z;
    }
}
template <int N, typename R>
__device__ __forceinline__ void link_mul(const RLink<N, R> &l, const Cx<R> (&h)[N], Cx<R> (&o)[N])
{
#pragma unroll
    for (int i = 0; i < N; i++) {
        Cx<R> z{l.r[i][0] * h[0].re, l.r[i][0] * h[0].im};
#pragma unroll
        for (int j = 1; j < N; j++) z = Cx<R>{fmadd(l.r[i][j], h[j].re, z.re), fmadd(l.r[i][j], h[j].im, z.im)};
        o[i] = z;
    }
}
template <int N, typename R>
__device__ __forceinline__ void link_mul_dag(const RLink<N, R> &l, const Cx<R> (&h)[N], Cx<R> (&o)[N])
{
#pragma unroll
    for (int i = 0; i < N; i++) {
        Cx<R> z{l.r[0][i] * h[0].re, l.r[0][i] * h[0].im};
#pragma unroll
        for (int j = 1; j < N; j++) z = Cx<R>{fmadd(l.r[j][i], h[j].re, z.re), fmadd(l.r[j][i], h[j].im, z.im)};
        o[i] = z;
    }
}

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
        o[i] = Cx<R>{fmadd(l.r[i][2], h[2].re, fmadd(l.r[i][1], h[1].re, l.r[i][0] * h[0].re)),
                     fmadd(l.r[i][2], h[2].im, fmadd(l.r[i][1], h[1].im, l.r[i][0] * h[0].im))};
}
template <typename R>
__device__ __forceinline__ void link_mul_dag(const AdjLink<R> &l, const Cx<R> (&h)[3], Cx<R> (&o)[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
        o[i] = Cx<R>{fmadd(l.r[2][i], h[2].re, fmadd(l.r[1][i], h[1].re, l.r[0][i] * h[0].re)),
                     fmadd(l.r[2][i], h[2].im, fmadd(l.r[1][i], h[1].im, l.r[0][i] * h[0].im))};
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
