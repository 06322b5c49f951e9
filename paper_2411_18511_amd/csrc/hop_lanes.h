// Hopping stencil for SU(4) two-index symmetric links (CPLX10, 10 x 10
// complex) in FP64 with four lanes per site.
//
// With one thread per site the format needs a 40-component FP64 accumulator,
// both half spinors and a streamed link row at once, which spills.  The split
// is the one of the REAL8 kernel (hop_quad.h) for complex links: the colours
// are cut into Q = 2 groups of H = 5, and lane (k, g) of a site's four owns
// output spins k and 2 + k for the colours of group g.  Per direction a lane
// loads the two spins that component k of the projected half spinor needs,
// forms that component for all N colours, multiplies by the rows of U of its
// colours (forward) or by the matching halves of all rows of U (backward),
// and accumulates; the lower spin takes the partner component in directions
// 1 and 2, handed over by a lane shuffle.  Products and sums follow the
// one-thread kernel's order (dense_mul_rows, dense_mul_dag_rows).
//
// Link layout (FP64): one array of 16-byte planes per parity and direction,
// entry e = N i + j in plane e.  (The same split for REAL15 measured no
// faster than its one-thread kernel, with two or four colour groups.)
#pragma once

#include "hop.h"

namespace hrd {

namespace lanes {

template <int REP>
struct Fmt {
    static_assert(!is_real_dense(REP), "complex link formats");
    static constexpr int N = NCol<REP>::value;
    static constexpr int Q = 2;                                    // colour groups
    static constexpr int H = (N + Q - 1) / Q;                      // colours per group
    static constexpr int kLanes = 2 * Q;                           // lanes per site
    static constexpr int kPlanes = link_bytes(REP, HRD_F64) / 16;  // planes per link
    static constexpr int kSpinorPlanes = 4 * N;                    // complex components per site
};

__device__ __forceinline__ Cx<double> ld_c(const char *base, uint32_t voff)
{
    const vd2 v = ld16d<false>(base + voff);
    return Cx<double>{v.x, v.y};
}

template <int M>
__device__ __forceinline__ void fence(Cx<double> (&v)[M])
{
#pragma unroll
    for (int i = 0; i < M; i++) asm volatile("" : "+v"(v[i].re), "+v"(v[i].im)::"memory");
}

__device__ __forceinline__ Cx<double> sel_neg(bool neg, Cx<double> v) { return neg ? -v : v; }

// plane 0 of a site in a 64-site tile of an FP64 spinor block of NC planes,
// and the distance between its planes (32-bit byte offsets from the block
// start: lanes_covers keeps a parity block below 4 GiB)
struct SiteOff {
    uint32_t base, step;
};
template <int NC>
__device__ __forceinline__ SiteOff site_off(int Vh, int site)
{
    const int b0 = site & ~63;
    const int nb = Vh - b0 < 64 ? Vh - b0 : 64;
    return SiteOff{(uint32_t)b0 * (uint32_t)(NC * 16) + (uint32_t)(site - b0) * 16u, (uint32_t)nb * 16u};
}

// Component k of the upper half spinor of (1 + SIG g_MU) psi for all colours
// (the expressions of project() for component k).
template <int REP, int MU, int SIG>
__device__ __forceinline__ void project_k(const char *src, int Vh, int j, int k, Cx<double> (&h)[Fmt<REP>::N])
{
    constexpr int N = Fmt<REP>::N;
    const int par = (MU == 0 || MU == 3) ? k + 2 : 3 - k;
    bool neg;
    if constexpr (MU == 0) neg = SIG < 0;
    else if constexpr (MU == 1) neg = SIG > 0;
    else neg = (k == 0) == (SIG > 0);
    const SiteOff so = site_off<Fmt<REP>::kSpinorPlanes>(Vh, j);
    const uint32_t vo = so.base + (uint32_t)(k * N) * so.step;
    const uint32_t vp = so.base + (uint32_t)(par * N) * so.step;
#pragma unroll
    for (int c = 0; c < N; c++) {
        const Cx<double> po = ld_c(src, vo + (uint32_t)c * so.step);
        const Cx<double> pp = ld_c(src, vp + (uint32_t)c * so.step);
        const Cx<double> t = (MU == 1 || MU == 3) ? mul_i(pp) : pp;
        h[c] = neg ? po - t : po + t;
    }
}

// M consecutive entries of a link starting at entry e0 (runtime), one plane
// each, from the link block lb of (parity, direction): vs = site * 16,
// vstride = Vh * 16
template <int M>
__device__ __forceinline__ void entries_cplx(const char *lb, uint32_t vs, uint32_t vstride, int e0,
                                             Cx<double> (&e)[M])
{
#pragma unroll
    for (int m = 0; m < M; m++) {
        const vd2 x = ld16d<kNtLinks>(lb + (size_t)(e0 + m) * vstride + vs);
        e[m] = Cx<double>{x.x, x.y};
    }
}

// u[r] = sum_j U[i][j] h[j] for the rows i = H hf + r of this lane's colour
// group hf (rows past N repeat row N - 1 and are discarded by the caller)
template <int REP>
__device__ __forceinline__ void mul_rows(const char *lb, int Vh, int site, int hf,
                                         const Cx<double> (&h)[Fmt<REP>::N], Cx<double> (&u)[Fmt<REP>::H])
{
    using F = Fmt<REP>;
    constexpr int N = F::N;
    const uint32_t vs = (uint32_t)site * 16u, vstride = (uint32_t)Vh * 16u;
#pragma unroll
    for (int r = 0; r < F::H; r++) u[r] = Cx<double>{0, 0};
#pragma unroll
    for (int r = 0; r < F::H; r++) {
        int i = hf * F::H + r;
        i = i < N ? i : N - 1;
        Cx<double> e[N];
        entries_cplx<N>(lb, vs, vstride, N * i, e);
        Cx<double> z = cmul(e[0], h[0]);
#pragma unroll
        for (int b = 1; b < N; b++) z = cfma(e[b], h[b], z);
        u[r] = z;
        if (r % 2 == 1) fence(u);  // at most two rows in flight
    }
}

// u[r] = sum_J conj(U[J][i]) h[J] for the colours i = H hf + r of this lane's
// group hf (the group's part of every row streamed; entries past the end of
// a row are discarded)
template <int REP>
__device__ __forceinline__ void mul_dag_rows(const char *lb, int Vh, int site, int hf,
                                             const Cx<double> (&h)[Fmt<REP>::N], Cx<double> (&u)[Fmt<REP>::H])
{
    using F = Fmt<REP>;
    constexpr int N = F::N;
    constexpr int H = F::H;
    const uint32_t vs = (uint32_t)site * 16u, vstride = (uint32_t)Vh * 16u;
#pragma unroll
    for (int J = 0; J < N; J++) {
        Cx<double> e[H];
        entries_cplx<H>(lb, vs, vstride, N * J + H * hf, e);
#pragma unroll
        for (int r = 0; r < H; r++) u[r] = J == 0 ? cmulc(e[r], h[0]) : cfmac(e[r], h[J], u[r]);
        if (J % 4 == 3) fence(u);  // at most four parts of rows in flight
    }
}

// the same colours' other component k, from lane (1 - k, g) = lane xor Q
template <int Q>
__device__ __forceinline__ Cx<double> shfl_partner(Cx<double> v)
{
    return Cx<double>{__shfl_xor(v.re, Q, 64), __shfl_xor(v.im, Q, 64)};
}

// up += u ; lo (spin 2 + k) takes its term of the reconstruction
template <int MU, int SIG, int H, int Q>
__device__ __forceinline__ void reconstruct_k(int k, const Cx<double> (&u)[H], Cx<double> (&up)[H],
                                              Cx<double> (&lo)[H])
{
    Cx<double> ux[H];
    if constexpr (MU == 1 || MU == 2) {
#pragma unroll
        for (int i = 0; i < H; i++) ux[i] = shfl_partner<Q>(u[i]);
    }
#pragma unroll
    for (int i = 0; i < H; i++) {
        up[i] = up[i] + u[i];
        Cx<double> l;
        if constexpr (MU == 0) l = u[i];
        else if constexpr (MU == 1) l = mul_i(ux[i]);
        else if constexpr (MU == 2) l = sel_neg(k == 1, ux[i]);
        else l = sel_neg(k == 1, mul_i(u[i]));
        lo[i] = SIG > 0 ? lo[i] + l : lo[i] - l;
    }
}

template <int REP, int MU, bool DAG>
__device__ __forceinline__ void lanes_dir(const Geom &g, const Site &s, int idx, int p, const void *U,
                                          const char *src, int k, int hf, Cx<double> (&up)[Fmt<REP>::H],
                                          Cx<double> (&lo)[Fmt<REP>::H])
{
    using F = Fmt<REP>;
    constexpr int N = F::N;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const char *Ub = reinterpret_cast<const char *>(U);
    const size_t block = (size_t)g.Vh * F::kPlanes * 16;  // bytes of one (parity, direction) link block
    {
        const int j = nbr_fwd(g, s, MU);
        Cx<double> h[N], u[F::H];
        project_k<REP, MU, SF>(src, g.Vh, j, k, h);
        if (MU == 0 && s.x[0] == g.L[0] - 1) {
#pragma unroll
            for (int c = 0; c < N; c++) h[c] = -h[c];
        }
        fence(h);
        mul_rows<REP>(Ub + (size_t)(4 * p + MU) * block, g.Vh, idx, hf, h, u);
        reconstruct_k<MU, SF, F::H, F::Q>(k, u, up, lo);
    }
    dir_fence(up);
    dir_fence(lo);
    {
        const int j = nbr_bwd(g, s, MU);
        Cx<double> h[N], u[F::H];
        project_k<REP, MU, SB>(src, g.Vh, j, k, h);
        if (MU == 0 && s.x[0] == 0) {
#pragma unroll
            for (int c = 0; c < N; c++) h[c] = -h[c];
        }
        fence(h);
        mul_dag_rows<REP>(Ub + (size_t)(4 * (1 - p) + MU) * block, g.Vh, j, hf, h, u);
        reconstruct_k<MU, SB, F::H, F::Q>(k, u, up, lo);
    }
    dir_fence(up);
    dir_fence(lo);
}

}  // namespace lanes

constexpr int kLanesBlock = 256;  // threads per workgroup

// sites per workgroup (and per norm partial) of the kernel for REP
template <int REP>
constexpr int lanes_sites() { return kLanesBlock / lanes::Fmt<REP>::kLanes; }

// Same operation and arguments as hop_kernel<REP, double, DAG, HAS_A, NORM,
// false, RUPD, CLOV_NONE> for REP = CPLX10, on a grid of
// ceil(Vh / lanes_sites) workgroups of 256 threads (one norm partial per
// workgroup, the granularity the one-thread kernel of these formats keeps).
template <int REP, bool DAG, bool HAS_A, bool NORM, bool RUPD>
__global__ __launch_bounds__(kLanesBlock) void hop_lanes_kernel(HopArgs a)
{
    using namespace lanes;
    using F = Fmt<REP>;
    constexpr int N = F::N;
    constexpr int H = F::H;
    static_assert(lanes_sites<REP>() == hop_sites_per_block(REP, HRD_F64), "norm partial granularity");
    const Geom &g = a.g;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int p = a.parity;
    const int w = lb * lanes_sites<REP>() + (int)(threadIdx.x / F::kLanes);
    const int k = (int)(threadIdx.x / F::Q) & 1;
    const int hf = (int)(threadIdx.x % F::Q);
    double nrm = 0;
    if (w < g.Vh) {
        int idx;
        const Site s = slab_site(g, w, p, &idx);
        Cx<double> up[H], lo[H];
#pragma unroll
        for (int i = 0; i < H; i++) up[i] = lo[i] = Cx<double>{0, 0};
        lanes_dir<REP, 0, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        lanes_dir<REP, 1, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        lanes_dir<REP, 2, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        lanes_dir<REP, 3, DAG>(g, s, idx, p, a.U, a.src, k, hf, up, lo);
        // this lane's planes: spin k and spin 2 + k, colours H hf .. H hf + H - 1 (< N)
        const SiteOff si = site_off<F::kSpinorPlanes>(g.Vh, idx);
        const uint32_t vu = si.base + (uint32_t)(k * N + H * hf) * si.step;
        const uint32_t vl = si.base + (uint32_t)((2 + k) * N + H * hf) * si.step;
        const double cb = a.b;
        const double ca = a.a;
        char *dst = RUPD ? reinterpret_cast<char *>(a.r) : a.dst;
#pragma unroll
        for (int i = 0; i < 2 * H; i++) {
            const int r = i % H;
            if (H * hf + r >= N) continue;
            const uint32_t off = (i < H ? vu : vl) + (uint32_t)r * si.step;
            const Cx<double> acc = i < H ? up[r] : lo[r];
            Cx<double> o = cb * acc;
            if constexpr (HAS_A) o = axpby(ca, ld_c(a.self, off), cb, acc);
            if constexpr (RUPD) {
                const Cx<double> rv = ld_c(dst, off);
                o = Cx<double>{fmadd(-a.sc[S_ALPHA], o.re, rv.re), fmadd(-a.sc[S_ALPHA], o.im, rv.im)};
            }
            st16d<kNtStore>(dst + off, vd2{o.re, o.im});
            if constexpr (NORM || RUPD) nrm += o.re * o.re + o.im * o.im;
        }
    }
    if constexpr (NORM || RUPD) {
        const double t = block_sum<kLanesBlock>(nrm);
        if (threadIdx.x == 0) a.partials[lb] = t;
    }
}

// CPLX10 FP64 launches the four-lane kernel covers: single parity, every
// spinor parity block below 4 GiB (32-bit offsets); the others run the
// one-thread kernel, whose norm partials have the same granularity.
inline bool lanes_covers(int rep, bool full, int Vh)
{
    return !full && rep == HRD_CPLX10 && (long long)Vh * 4 * ncolour(rep) * 16 < (1ll << 32);
}

template <int REP>
hipError_t launch_hop_lanes(const HopArgs &a, bool dag, bool has_a, bool norm, hipStream_t st)
{
    const dim3 grid((a.g.Vh + lanes_sites<REP>() - 1) / lanes_sites<REP>()), block(kLanesBlock);
#define HRD_LANES(D, A, NR) hipLaunchKernelGGL((hop_lanes_kernel<REP, D, A, NR, false>), grid, block, 0, st, a)
    if (dag) {
        if (has_a) {
            if (norm) HRD_LANES(true, true, true);
            else HRD_LANES(true, true, false);
        } else {
            if (norm) HRD_LANES(true, false, true);
            else HRD_LANES(true, false, false);
        }
    } else {
        if (has_a) {
            if (norm) HRD_LANES(false, true, true);
            else HRD_LANES(false, true, false);
        } else {
            if (norm) HRD_LANES(false, false, true);
            else HRD_LANES(false, false, false);
        }
    }
#undef HRD_LANES
    return hipGetLastError();
}

template <int REP>
hipError_t launch_hop_lanes_rupdate(const HopArgs &a, hipStream_t st)
{
    const dim3 grid((a.g.Vh + lanes_sites<REP>() - 1) / lanes_sites<REP>()), block(kLanesBlock);
    hipLaunchKernelGGL((hop_lanes_kernel<REP, true, true, false, true>), grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace hrd
