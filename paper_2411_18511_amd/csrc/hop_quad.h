// Hopping stencil for SU(3) adjoint links (REAL8, 8 x 8 real) in FP64 with
// four lanes per site.
//
// The one-thread-per-site kernel keeps a 32-component FP64 accumulator and
// whole neighbour spinors in registers and runs at one wave per SIMD.  Here
// lane (k, h) of a site's quad owns the output spins k (upper) and 2 + k
// (lower) for the colours of half h (4h .. 4h + 3): per direction it loads
// only the two spins that component k of the projected half spinor needs
// (spin k and its partner), projects, multiplies by its four rows of U (or
// the matching half rows of U^T) and accumulates.  The lower spin 2 + k takes
// the other component in directions 1 and 2, which the partner lane (1 - k, h)
// hands over by a lane shuffle.  Every output component is formed by the same
// operations in the same order as in the one-thread kernel (signs and partner
// spins are chosen by selects, which are exact), so the results are identical.
#pragma once

#include "hop.h"

namespace hrd {

constexpr int kQuadBlock = 4 * kHopBlock;  // threads per workgroup: kHopBlock sites

namespace quad {

constexpr int N = 8;           // colours of the representation
constexpr int kRowPlanes = 4;  // 16-byte planes (two doubles) per link row
constexpr int kPlanes = 32;    // planes per link

// Loads address a wave-uniform base plus a 32-bit per-lane byte offset, so
// each load needs no 64-bit address of its own.  One parity of a REAL8 FP64
// spinor or link direction then has to stay below 4 GiB (quad_covers).
__device__ __forceinline__ Cx<double> ld_c(const char *ubase, uint32_t voff)
{
    const vd2 v = ld16d<false>(ubase + voff);
    return Cx<double>{v.x, v.y};
}

// Compiler fence on a register array: the loads after it are not hoisted
// above the work before it, which bounds the live registers of a direction.
template <int M>
__device__ __forceinline__ void fence(Cx<double> (&v)[M])
{
#pragma unroll
    for (int i = 0; i < M; i++) asm volatile("" : "+v"(v[i].re), "+v"(v[i].im)::"memory");
}

__device__ __forceinline__ Cx<double> sel_neg(bool neg, Cx<double> v) { return neg ? -v : v; }

// A site in a 64-site tile of a REAL8 FP64 spinor block (32 planes): byte
// offset of its plane 0 and the distance between its planes (32-bit; plane q
// at base + q step, the offsets of tile_off).
struct SiteOff {
    uint32_t base, step;
};
__device__ __forceinline__ SiteOff site_off(int Vh, int site)
{
    const int b0 = site & ~63;
    const int nb = Vh - b0 < 64 ? Vh - b0 : 64;
    return SiteOff{(uint32_t)b0 * 512u + (uint32_t)(site - b0) * 16u, (uint32_t)nb * 16u};
}

// Component k of the upper half spinor of (1 + SIG g_MU) psi (the expressions
// of project(), with the spin pairing and signs of component k).
template <int MU, int SIG>
__device__ __forceinline__ void project_k(const char *src, int Vh, int j, int k, Cx<double> (&h)[N])
{
    const int par = (MU == 0 || MU == 3) ? k + 2 : 3 - k;
    // h = p_k + (s) t, t = p_par (MU 0, 2) or i p_par (MU 1, 3)
    bool neg;
    if constexpr (MU == 0) neg = SIG < 0;
    else if constexpr (MU == 1) neg = SIG > 0;
    else neg = (k == 0) == (SIG > 0);  // MU 2, 3: component 0 subtracts for SIG > 0
    const SiteOff so = site_off(Vh, j);
    const uint32_t vo = so.base + (uint32_t)(k * N) * so.step;
    const uint32_t vp = so.base + (uint32_t)(par * N) * so.step;
    Cx<double> po[N], pp[N];
#pragma unroll
    for (int c = 0; c < N; c++) {
        po[c] = ld_c(src, vo + (uint32_t)c * so.step);
        pp[c] = ld_c(src, vp + (uint32_t)c * so.step);
    }
#pragma unroll
    for (int c = 0; c < N; c++) {
        const Cx<double> t = (MU == 1 || MU == 3) ? mul_i(pp[c]) : pp[c];
        h[c] = neg ? po[c] - t : po[c] + t;
    }
}

// u[i] = sum_b U[4hf + i][b] h[b] (rows streamed, row-wise FMA order of
// dense_mul_rows); lb: the link block of (parity, direction)
__device__ __forceinline__ void mul_rows(const char *lb, int Vh, int site, int hf, const Cx<double> (&h)[N],
                                         Cx<double> (&u)[4])
{
    const uint32_t vo = ((uint32_t)(4 * hf * kRowPlanes) * (uint32_t)Vh + (uint32_t)site) * 16u;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        double e[N];
#pragma unroll
        for (int q = 0; q < kRowPlanes; q++) {
            const vd2 v = ld16d<kNtLinks>(lb + (size_t)(i * kRowPlanes + q) * Vh * 16 + vo);
            e[2 * q] = v.x;
            e[2 * q + 1] = v.y;
        }
        Cx<double> z{e[0] * h[0].re, e[0] * h[0].im};
#pragma unroll
        for (int b = 1; b < N; b++) z = Cx<double>{fmadd(e[b], h[b].re, z.re), fmadd(e[b], h[b].im, z.im)};
        u[i] = z;
    }
}

// u[i] = sum_J U[J][4hf + i] h[J] (half rows streamed, order of
// dense_mul_dag_rows)
__device__ __forceinline__ void mul_dag_rows(const char *lb, int Vh, int site, int hf, const Cx<double> (&h)[N],
                                             Cx<double> (&u)[4])
{
    const uint32_t vo = ((uint32_t)(2 * hf) * (uint32_t)Vh + (uint32_t)site) * 16u;
#pragma unroll
    for (int J = 0; J < N; J++) {
        double e[4];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const vd2 v = ld16d<kNtLinks>(lb + (size_t)(J * kRowPlanes + q) * Vh * 16 + vo);
            e[2 * q] = v.x;
            e[2 * q + 1] = v.y;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if (J == 0) u[i] = Cx<double>{e[i] * h[0].re, e[i] * h[0].im};
            else u[i] = Cx<double>{fmadd(e[i], h[J].re, u[i].re), fmadd(e[i], h[J].im, u[i].im)};
        }
        if (J == 3) fence(u);  // at most four half rows in flight
    }
}

__device__ __forceinline__ Cx<double> shfl_partner(Cx<double> v)
{
    return Cx<double>{__shfl_xor(v.re, 2, 64), __shfl_xor(v.im, 2, 64)};
}

// acc_up += u ; acc_lo (spin 2 + k) += or -= its term of the reconstruction
template <int MU, int SIG>
__device__ __forceinline__ void reconstruct_k(int k, const Cx<double> (&u)[4], Cx<double> (&up)[4],
                                              Cx<double> (&lo)[4])
{
    Cx<double> ux[4];
    if constexpr (MU == 1 || MU == 2) {
#pragma unroll
        for (int i = 0; i < 4; i++) ux[i] = shfl_partner(u[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        up[i] = up[i] + u[i];
        // lower term of spin 2 + k: MU 0: +u_k; 1: i u_(1-k); 2: +u_1 (spin 2) / -u_0 (spin 3);
        // 3: i u_0 (spin 2) / -i u_1 (spin 3)
        Cx<double> l;
        if constexpr (MU == 0) l = u[i];
        else if constexpr (MU == 1) l = mul_i(ux[i]);
        else if constexpr (MU == 2) l = sel_neg(k == 1, ux[i]);
        else l = sel_neg(k == 1, mul_i(u[i]));
        lo[i] = SIG > 0 ? lo[i] + l : lo[i] - l;
    }
}

template <int MU, bool DAG>
__device__ __forceinline__ void quad_dir(const Geom &g, const Site &s, int idx, int p, const void *U, const char *src,
                                         int k, int hf, Cx<double> (&up)[4], Cx<double> (&lo)[4])
{
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const char *Ub = reinterpret_cast<const char *>(U);
    {
        const int j = nbr_fwd(g, s, MU);
        Cx<double> h[N], u[4];
        project_k<MU, SF>(src, g.Vh, j, k, h);
        if (MU == 0 && s.x[0] == g.L[0] - 1) {
#pragma unroll
            for (int c = 0; c < N; c++) h[c] = -h[c];
        }
        fence(h);
        mul_rows(Ub + (size_t)(4 * p + MU) * g.Vh * kPlanes * 16, g.Vh, idx, hf, h, u);
        reconstruct_k<MU, SF>(k, u, up, lo);
    }
    dir_fence(up);
    dir_fence(lo);
    {
        const int j = nbr_bwd(g, s, MU);
        Cx<double> h[N], u[4];
        project_k<MU, SB>(src, g.Vh, j, k, h);
        if (MU == 0 && s.x[0] == 0) {
#pragma unroll
            for (int c = 0; c < N; c++) h[c] = -h[c];
        }
        fence(h);
        mul_dag_rows(Ub + (size_t)(4 * (1 - p) + MU) * g.Vh * kPlanes * 16, g.Vh, j, hf, h, u);
        reconstruct_k<MU, SB>(k, u, up, lo);
    }
    dir_fence(up);
    dir_fence(lo);
}

}  // namespace quad

// Same operation and arguments as hop_kernel<HRD_REAL8, double, DAG, HAS_A,
// NORM, false, RUPD, CLOV_NONE>, on a grid of hop_blocks(g) workgroups of
// kQuadBlock threads (the NORM partials keep one entry per kHopBlock sites).
template <bool DAG, bool HAS_A, bool NORM, bool RUPD>
__global__ __launch_bounds__(kQuadBlock) void hop_quad_kernel(HopArgs a)
{
    using namespace quad;
    const Geom &g = a.g;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int p = a.parity;
    const int w = lb * kHopBlock + (int)(threadIdx.x >> 2);
    const int k = (threadIdx.x >> 1) & 1;
    const int hf = threadIdx.x & 1;
    double nrm = 0;
    if (w < g.Vh) {
        int idx;
        const Site s = slab_site(g, w, p, &idx);
        Cx<double> up[4], lo[4];
#pragma unroll
        for (int i = 0; i < 4; i++) up[i] = lo[i] = Cx<double>{0, 0};
        quad_dir<0, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        quad_dir<1, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        quad_dir<2, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        quad_dir<3, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        // this lane's planes: spin k and spin 2 + k, colours 4 hf .. 4 hf + 3
        const int pu = k * N + 4 * hf, pl = (2 + k) * N + 4 * hf;
        const SiteOff si = site_off(g.Vh, idx);
        const uint32_t vu = si.base + (uint32_t)pu * si.step;
        const uint32_t vl = si.base + (uint32_t)pl * si.step;
        const double cb = a.b;
        Cx<double> out[8];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            out[i] = cb * up[i];
            out[4 + i] = cb * lo[i];
        }
        if constexpr (HAS_A) {
            const double ca = a.a;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                out[i] = axpby(ca, ld_c(a.self, vu + (uint32_t)i * si.step), cb, up[i]);
                out[4 + i] = axpby(ca, ld_c(a.self, vl + (uint32_t)i * si.step), cb, lo[i]);
            }
        }
        char *dst = RUPD ? reinterpret_cast<char *>(a.r) : a.dst;
        if constexpr (RUPD) {
            const double alpha = a.sc[S_ALPHA];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const Cx<double> rv = ld_c(dst, (i < 4 ? vu : vl) + (uint32_t)(i & 3) * si.step);
                out[i] = Cx<double>{fmadd(-alpha, out[i].re, rv.re), fmadd(-alpha, out[i].im, rv.im)};
            }
        }
#pragma unroll
        for (int i = 0; i < 8; i++) {
            st16d<kNtStore>(dst + ((i < 4 ? vu : vl) + (uint32_t)(i & 3) * si.step), vd2{out[i].re, out[i].im});
            if constexpr (NORM || RUPD) nrm += out[i].re * out[i].re + out[i].im * out[i].im;
        }
    }
    if constexpr (NORM || RUPD) {
        const double t = block_sum<kQuadBlock>(nrm);
        if (threadIdx.x == 0) a.partials[lb] = t;
    }
}

// REAL8 / FP64 launches that the quad kernel covers (single parity, no
// clover); returns false when the one-thread kernel has to run.
inline bool quad_covers(int rep, bool full, int Vh)
{
    return rep == HRD_REAL8 && !full && (long long)Vh * 512 < (1ll << 32);
}

inline hipError_t launch_hop_quad(const HopArgs &a, bool dag, bool has_a, bool norm, hipStream_t st)
{
    const dim3 grid(hop_blocks(a.g)), block(kQuadBlock);
#define HRD_QUAD(D, A, NR) hipLaunchKernelGGL((hop_quad_kernel<D, A, NR, false>), grid, block, 0, st, a)
    if (dag) {
        if (has_a) {
            if (norm) HRD_QUAD(true, true, true);
            else HRD_QUAD(true, true, false);
        } else {
            if (norm) HRD_QUAD(true, false, true);
            else HRD_QUAD(true, false, false);
        }
    } else {
        if (has_a) {
            if (norm) HRD_QUAD(false, true, true);
            else HRD_QUAD(false, true, false);
        } else {
            if (norm) HRD_QUAD(false, false, true);
            else HRD_QUAD(false, false, false);
        }
    }
#undef HRD_QUAD
    return hipGetLastError();
}

inline hipError_t launch_hop_quad_rupdate(const HopArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((hop_quad_kernel<true, true, false, true>), dim3(hop_blocks(a.g)), dim3(kQuadBlock), 0, st,
                       a);
    return hipGetLastError();
}

}  // namespace hrd
