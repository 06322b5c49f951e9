// Hopping-kernel templates shared by the translation units that instantiate
// them for the SU(2) link formats (dslash.hip) and the dense SU(N > 2)
// formats (dslash_sun.hip).
// Wilson hopping stencil on one parity (the "inner Dirac kernel" of the
// paper's Sec. 2.1, here covering the whole single-GPU lattice), with fused
// epilogues for the plain operator D = m - H/2, the off-diagonal blocks
// D_eo = -H_eo/2 and the second stage of the even/odd operator
// D^ = m - (1/m) D_eo D_oe, and the clover variants (site matrix M = m + A
// in place of m: D = M - H/2, D^ = M_ee - D_eo M_oo^{-1} D_oe).
//
// One thread per target site.  For each of the 8 directions the neighbour
// spinor (opposite parity) is spin-projected to a half spinor with
// (1 -+ g_mu), multiplied by U or U^+ on colour, and the lower two spin
// components are reconstructed from the upper two (the projector has rank 2).
// Every link is read exactly once per hop; the sign s_mu(x) of the
// time-antiperiodic boundary is applied to the half spinor.
#pragma once

#include "clover.h"
#include "kernels.h"
#include "spin.h"

namespace hrd {

// Cache policy of the hopping kernel (measured on MI355X; the workgroup size
// is hop_block below): links and outputs are used once per hop and go
// through non-temporal loads and stores, except in the one-launch plain
// operator, where every link serves one even and one odd target and the
// blocks of the two parities at the same position run side by side on one
// XCD (temporal link loads).
constexpr bool kNtLinks = true;
constexpr bool kNtLinksFull = false;
constexpr bool kNtStore = true;

constexpr int kHopBlock = 256;  // threads per workgroup, and sites per norm partial

// Workgroup size of one instantiation (hop_sites_per_block).  The FP64
// kernels of the SU(2) formats hold one wave per SIMD and run one-wave
// workgroups, so each SIMD starts its next workgroup as soon as its own wave
// ends instead of waiting for the slowest of four (48^4 FP64 hop
// 394 -> 381 us, plain D 739 -> 716 us); norm partials follow the workgroups.
template <int REP, typename S>
constexpr int hop_block()
{
    return hop_sites_per_block(REP, std::is_same<S, double>::value ? HRD_F64 : HRD_F32);
}
static_assert(hop_sites_per_block(HRD_FUND, HRD_F32) == kHopBlock, "hop workgroup sizes");

namespace {

// Barrier between the direction terms of the dense formats: the accumulator
// is pinned in registers (each component passes through an empty asm
// statement) and memory operations are ordered, so one direction's products
// are finished before the next direction's loads issue.  Without it the
// compiler issues the loads of all eight terms first and defers their
// arithmetic, which needs the spinors and links of every term live at once.
template <typename R, int NC>
__device__ __forceinline__ void dir_fence(Cx<R> (&acc)[NC])
{
#pragma unroll
    for (int k = 0; k < NC; k++) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im)::"memory");
}

// S: storage type of the source spinor and the links; R: arithmetic type.
template <int MU, bool DAG, int REP, typename S, bool NTL = kNtLinks, bool REL = false,
          typename R = typename Arith<S>::type>
__device__ __forceinline__ void hop_dir(const Geom &g, const Site &s, int idx, int p, const void *U,
                                        const char *src, Cx<R> (&acc)[4 * NCol<REP>::value])
{
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    constexpr int SF = DAG ? +1 : -1;  // forward term uses (1 + SF g_mu)
    constexpr int SB = -SF;            // backward term uses (1 + SB g_mu)
    using IO = SpinorIO<S>;
    using LIO = LinkIO<REP, S>;
    {
        const int j = nbr_fwd(g, s, MU);
        Cx<R> psi[NC];
        IO::template load<NC, false, REL>(src, g.Vh, j, psi);
        const auto l = LIO::template load<NTL, REL>(U, g.Vh, p, MU, idx);
        Cx<R> h0[N], h1[N], u0[N], u1[N];
        project<MU, SF, N, R>(psi, h0, h1);
        if (MU == 0 && s.x[0] == g.L[0] - 1) {
#pragma unroll
            for (int c = 0; c < N; c++) {
                h0[c] = -h0[c];
                h1[c] = -h1[c];
            }
        }
        link_mul(l, h0, u0);
        link_mul(l, h1, u1);
        reconstruct<MU, SF, N, R>(acc, u0, u1);
    }
    {
        const int j = nbr_bwd(g, s, MU);
        Cx<R> psi[NC];
        IO::template load<NC, false, REL>(src, g.Vh, j, psi);
        const auto l = LIO::template load<NTL, REL>(U, g.Vh, 1 - p, MU, j);
        Cx<R> h0[N], h1[N], u0[N], u1[N];
        project<MU, SB, N, R>(psi, h0, h1);
        if (MU == 0 && s.x[0] == 0) {
#pragma unroll
            for (int c = 0; c < N; c++) {
                h0[c] = -h0[c];
                h1[c] = -h1[c];
            }
        }
        link_mul_dag(l, h0, u0);
        link_mul_dag(l, h1, u1);
        reconstruct<MU, SB, N, R>(acc, u0, u1);
    }
}

// Row r of a dense link: the colour products stream the link one row at a
// time, so an N x N link never has to be live in registers at once.
template <int REP, typename S, int I, typename T, int N>
__device__ __forceinline__ void dense_row(const void *U, int Vh, int p, int mu, int site, T (&row)[N])
{
    LinkIO<REP, S>::template load_row<I, kNtLinks>(U, Vh, p, mu, site, row);
}

template <typename R>
__device__ __forceinline__ Cx<R> row_entry(const Cx<R> &e) { return e; }
template <typename R>
__device__ __forceinline__ Cx<R> row_entry(const R &e) { return Cx<R>{e, R(0)}; }

// o = U h0, U h1 (rows streamed)
template <int REP, typename S, int I, int N, typename R>
__device__ __forceinline__ void dense_mul_rows(const void *U, int Vh, int p, int mu, int site, const Cx<R> (&h0)[N],
                                               const Cx<R> (&h1)[N], Cx<R> (&o0)[N], Cx<R> (&o1)[N])
{
    if constexpr (I < N) {
        using Row = std::conditional_t<is_real_dense(REP), R, Cx<R>>;
        Row row[N];
        dense_row<REP, S, I>(U, Vh, p, mu, site, row);
        if constexpr (is_real_dense(REP)) {
            Cx<R> z0{row[0] * h0[0].re, row[0] * h0[0].im}, z1{row[0] * h1[0].re, row[0] * h1[0].im};
#pragma unroll
            for (int j = 1; j < N; j++) {
                z0 = Cx<R>{fmadd(row[j], h0[j].re, z0.re), fmadd(row[j], h0[j].im, z0.im)};
                z1 = Cx<R>{fmadd(row[j], h1[j].re, z1.re), fmadd(row[j], h1[j].im, z1.im)};
            }
            o0[I] = z0;
            o1[I] = z1;
        } else {
            Cx<R> z0 = cmul(row[0], h0[0]), z1 = cmul(row[0], h1[0]);
#pragma unroll
            for (int j = 1; j < N; j++) {
                z0 = cfma(row[j], h0[j], z0);
                z1 = cfma(row[j], h1[j], z1);
            }
            o0[I] = z0;
            o1[I] = z1;
        }
        dense_mul_rows<REP, S, I + 1, N, R>(U, Vh, p, mu, site, h0, h1, o0, o1);
    }
}

// o += U^+ h0, U^+ h1 with row J of U contributing conj(U_J i) h_J to o_i
template <int REP, typename S, int J, int N, typename R>
__device__ __forceinline__ void dense_mul_dag_rows(const void *U, int Vh, int p, int mu, int site,
                                                   const Cx<R> (&h0)[N], const Cx<R> (&h1)[N], Cx<R> (&o0)[N],
                                                   Cx<R> (&o1)[N])
{
    if constexpr (J < N) {
        using Row = std::conditional_t<is_real_dense(REP), R, Cx<R>>;
        Row row[N];
        dense_row<REP, S, J>(U, Vh, p, mu, site, row);
#pragma unroll
        for (int i = 0; i < N; i++) {
            if constexpr (is_real_dense(REP)) {
                if (J == 0) {
                    o0[i] = Cx<R>{row[i] * h0[0].re, row[i] * h0[0].im};
                    o1[i] = Cx<R>{row[i] * h1[0].re, row[i] * h1[0].im};
                } else {
                    o0[i] = Cx<R>{fmadd(row[i], h0[J].re, o0[i].re), fmadd(row[i], h0[J].im, o0[i].im)};
                    o1[i] = Cx<R>{fmadd(row[i], h1[J].re, o1[i].re), fmadd(row[i], h1[J].im, o1[i].im)};
                }
            } else {
                if (J == 0) {
                    o0[i] = cmulc(row[i], h0[0]);
                    o1[i] = cmulc(row[i], h1[0]);
                } else {
                    o0[i] = cfmac(row[i], h0[J], o0[i]);
                    o1[i] = cfmac(row[i], h1[J], o1[i]);
                }
            }
        }
        dense_mul_dag_rows<REP, S, J + 1, N, R>(U, Vh, p, mu, site, h0, h1, o0, o1);
    }
}

// Dense links of at most 128 bytes (CPLX3 and CPLX4 in F16 and FP32) are
// loaded whole and multiplied from registers (link_mul: the same operations
// in the same order as the row-streamed products), so their few loads are
// issued together and a plane shared by two rows is read once (32^4 SU(3)
// fundamental FP32 hop 87.0 -> 84.4 us, D^ 177 -> 170 us).
template <int REP, typename S>
constexpr bool dense_whole_link()
{
    constexpr int prec = std::is_same<S, double>::value ? HRD_F64 : std::is_same<S, float>::value ? HRD_F32 : HRD_F16;
    return is_dense(REP) && !is_real_dense(REP) && REP != HRD_SU3_ROW2 && link_bytes(REP, prec) <= 128;
}

// One direction of the stencil for the dense formats (same arithmetic as
// hop_dir, links streamed by row or, for small links, loaded whole).
template <int MU, bool DAG, int REP, typename S, typename R = typename Arith<S>::type>
__device__ __forceinline__ void hop_dir_dense(const Geom &g, const Site &s, int idx, int p, const void *U,
                                              const char *src, Cx<R> (&acc)[4 * NCol<REP>::value])
{
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    using IO = SpinorIO<S>;
    {
        const int j = nbr_fwd(g, s, MU);
        Cx<R> h0[N], h1[N], u0[N], u1[N];
        {
            Cx<R> psi[NC];
            IO::template load<NC>(src, g.Vh, j, psi);
            project<MU, SF, N, R>(psi, h0, h1);
        }
        if (MU == 0 && s.x[0] == g.L[0] - 1) {
#pragma unroll
            for (int c = 0; c < N; c++) {
                h0[c] = -h0[c];
                h1[c] = -h1[c];
            }
        }
        if constexpr (dense_whole_link<REP, S>()) {
            const auto l = LinkIO<REP, S>::template load<kNtLinks>(U, g.Vh, p, MU, idx);
            link_mul(l, h0, u0);
            link_mul(l, h1, u1);
        } else {
            dense_mul_rows<REP, S, 0, N, R>(U, g.Vh, p, MU, idx, h0, h1, u0, u1);
        }
        reconstruct<MU, SF, N, R>(acc, u0, u1);
    }
    dir_fence(acc);
    {
        const int j = nbr_bwd(g, s, MU);
        Cx<R> h0[N], h1[N], u0[N], u1[N];
        {
            Cx<R> psi[NC];
            IO::template load<NC>(src, g.Vh, j, psi);
            project<MU, SB, N, R>(psi, h0, h1);
        }
        if (MU == 0 && s.x[0] == 0) {
#pragma unroll
            for (int c = 0; c < N; c++) {
                h0[c] = -h0[c];
                h1[c] = -h1[c];
            }
        }
        if constexpr (dense_whole_link<REP, S>()) {
            const auto l = LinkIO<REP, S>::template load<kNtLinks>(U, g.Vh, 1 - p, MU, j);
            link_mul_dag(l, h0, u0);
            link_mul_dag(l, h1, u1);
        } else {
            dense_mul_dag_rows<REP, S, 0, N, R>(U, g.Vh, 1 - p, MU, j, h0, h1, u0, u1);
        }
        reconstruct<MU, SB, N, R>(acc, u0, u1);
    }
    dir_fence(acc);
}

// out = a psi_self(x) + b (H psi_src)(x) on the target parity; FULL runs both
// parities in one launch (blocks alternate parity), NORM writes one partial
// of ||out||^2 per block.  CLOV selects a clover epilogue (CloverMode).
// S is the storage type of the operator's spinors and links (double, float or
// h16), R = Arith<S>::type the arithmetic; the residual of the RUPD epilogue
// and the clover fields are stored in R.
template <int REP, typename S, bool DAG, bool HAS_A, bool NORM, bool FULL, bool RUPD, int CLOV, bool REL>
__device__ __forceinline__ void hop_body(const HopArgs &a)
{
    using R = typename Arith<S>::type;
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    const Geom &g = a.g;
    int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int part_idx = lb;
    int p;
    const char *src;
    const char *self;
    char *dst;
    if constexpr (FULL) {
        p = lb & 1;
        lb >>= 1;
        src = a.src + (size_t)(1 - p) * a.half_bytes;
        self = a.src + (size_t)p * a.half_bytes;
        dst = a.dst + (size_t)p * a.half_bytes;
    } else {
        p = a.parity;
        src = a.src;
        self = a.self;
        dst = a.dst;
    }
    const int w = lb * hop_block<REP, S>() + threadIdx.x;
    double nrm = 0;
    if (w < g.Vh) {
        int idx;
        const Site s = slab_site(g, w, p, &idx);
        Cx<R> acc[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) acc[k] = Cx<R>{0, 0};
        if constexpr (is_dense(REP)) {
            hop_dir_dense<0, DAG, REP, S>(g, s, idx, p, a.U, src, acc);
            hop_dir_dense<1, DAG, REP, S>(g, s, idx, p, a.U, src, acc);
            hop_dir_dense<2, DAG, REP, S>(g, s, idx, p, a.U, src, acc);
            hop_dir_dense<3, DAG, REP, S>(g, s, idx, p, a.U, src, acc);
        } else {
            constexpr bool NTL = FULL ? kNtLinksFull : kNtLinks;
            hop_dir<0, DAG, REP, S, NTL, REL>(g, s, idx, p, a.U, src, acc);
            hop_dir<1, DAG, REP, S, NTL, REL>(g, s, idx, p, a.U, src, acc);
            hop_dir<2, DAG, REP, S, NTL, REL>(g, s, idx, p, a.U, src, acc);
            hop_dir<3, DAG, REP, S, NTL, REL>(g, s, idx, p, a.U, src, acc);
        }
        const R cb = (R)a.b;
        Cx<R> out[NC];
        if constexpr (CLOV == CLOV_INV) {
            Cx<R> t[NC];
#pragma unroll
            for (int k = 0; k < NC; k++) t[k] = cb * acc[k];
            clover_apply<N, R, kNtLinks>(a.clov, g.Vh, p, idx, t, out);
        } else if constexpr (HAS_A && CLOV == CLOV_SELF) {
            Cx<R> self_v[NC], ms[NC];
            SpinorIO<S>::template load<NC>(self, g.Vh, idx, self_v);
            clover_apply<N, R, kNtLinks>(a.clov, g.Vh, p, idx, self_v, ms);
#pragma unroll
            for (int k = 0; k < NC; k++)
                out[k] = Cx<R>{fmadd(cb, acc[k].re, ms[k].re), fmadd(cb, acc[k].im, ms[k].im)};
        } else if constexpr (HAS_A) {
            const R ca = (R)a.a;
            Cx<R> self_v[NC];
            SpinorIO<S>::template load<NC>(self, g.Vh, idx, self_v);
#pragma unroll
            for (int k = 0; k < NC; k++) out[k] = axpby(ca, self_v[k], cb, acc[k]);
        } else {
#pragma unroll
            for (int k = 0; k < NC; k++) out[k] = cb * acc[k];
        }
        if constexpr (RUPD) {
            // r <- r - alpha out ; out (= A p) itself is never written
            const R alpha = (R)a.sc[S_ALPHA];
            Cx<R> rv[NC];
            SpinorIO<R>::template load<NC>(a.r, g.Vh, idx, rv);
#pragma unroll
            for (int k = 0; k < NC; k++) {
                rv[k] = Cx<R>{fmadd(-alpha, out[k].re, rv[k].re), fmadd(-alpha, out[k].im, rv[k].im)};
                nrm += (double)rv[k].re * (double)rv[k].re + (double)rv[k].im * (double)rv[k].im;
            }
            SpinorIO<R>::template store<NC, kNtStore>(a.r, g.Vh, idx, rv);
        } else {
            SpinorIO<S>::template store<NC, kNtStore>(dst, g.Vh, idx, out);
            if constexpr (NORM) {
#pragma unroll
                for (int k = 0; k < NC; k++)
                    nrm += (double)out[k].re * (double)out[k].re + (double)out[k].im * (double)out[k].im;
            }
        }
    }
    if constexpr (NORM) {
        const double t = block_sum<hop_block<REP, S>()>(nrm);
        if (threadIdx.x == 0) a.partials[part_idx] = t;
    }
}

template <int REP, typename S, bool DAG, bool HAS_A, bool NORM, bool FULL, bool RUPD = false, int CLOV = CLOV_NONE,
          bool REL = false>
__global__ __launch_bounds__((hop_block<REP, S>())) void hop_kernel(HopArgs a)
{
    hop_body<REP, S, DAG, HAS_A, NORM, FULL, RUPD, CLOV, REL>(a);
}

// FP64 SU(2) formats take the kernel with 32-bit-offset loads when the host
// has found every block below 2 GiB (HopArgs::rel), else 64-bit addresses.
// A single kernel holding both paths behind a uniform branch measured slower
// than either.
template <int REP, typename S, bool DAG, bool HAS_A, bool NORM, bool FULL, bool RUPD, int CLOV>
void launch_hop_kernel(const HopArgs &a, hipStream_t st)
{
    constexpr int blk = hop_block<REP, S>();
    const dim3 grid(((a.g.Vh + blk - 1) / blk) * (FULL ? 2 : 1));
    if constexpr (std::is_same<S, double>::value && !is_dense(REP)) {
        if (a.rel) {
            hipLaunchKernelGGL((hop_kernel<REP, S, DAG, HAS_A, NORM, FULL, RUPD, CLOV, true>), grid, dim3(blk), 0, st,
                               a);
            return;
        }
    }
    hipLaunchKernelGGL((hop_kernel<REP, S, DAG, HAS_A, NORM, FULL, RUPD, CLOV, false>), grid, dim3(blk), 0, st, a);
}

template <int REP, typename S, int CLOV>
hipError_t dispatch_hop(const HopArgs &a, bool dag, bool has_a, bool norm, bool full, hipStream_t st)
{
#define HRD_LAUNCH(D, A, NR, F) launch_hop_kernel<REP, S, D, A, NR, F, false, CLOV>(a, st)
    if constexpr (CLOV == CLOV_INV) {
        // M^{-1} (b H src): no self term, no norm
        if (dag) HRD_LAUNCH(true, false, false, false);
        else HRD_LAUNCH(false, false, false, false);
    } else if constexpr (CLOV == CLOV_SELF) {
        if (full) {
            if (dag) HRD_LAUNCH(true, true, false, true);
            else HRD_LAUNCH(false, true, false, true);
        } else if (dag) {
            if (norm) HRD_LAUNCH(true, true, true, false);
            else HRD_LAUNCH(true, true, false, false);
        } else {
            if (norm) HRD_LAUNCH(false, true, true, false);
            else HRD_LAUNCH(false, true, false, false);
        }
    } else if (full) {
        if (dag)
            HRD_LAUNCH(true, true, false, true);
        else
            HRD_LAUNCH(false, true, false, true);
    } else if (dag) {
        if (has_a) {
            if (norm) HRD_LAUNCH(true, true, true, false);
            else HRD_LAUNCH(true, true, false, false);
        } else {
            if (norm) HRD_LAUNCH(true, false, true, false);
            else HRD_LAUNCH(true, false, false, false);
        }
    } else {
        if (has_a) {
            if (norm) HRD_LAUNCH(false, true, true, false);
            else HRD_LAUNCH(false, true, false, false);
        } else {
            if (norm) HRD_LAUNCH(false, false, true, false);
            else HRD_LAUNCH(false, false, false, false);
        }
    }
#undef HRD_LAUNCH
    return hipGetLastError();
}

template <int REP, typename S>
hipError_t dispatch_hop_clov(const HopArgs &a, bool dag, bool has_a, bool norm, bool full, hipStream_t st, int clov)
{
    switch (clov) {
        case CLOV_SELF: return dispatch_hop<REP, S, CLOV_SELF>(a, dag, has_a, norm, full, st);
        case CLOV_INV: return dispatch_hop<REP, S, CLOV_INV>(a, dag, has_a, norm, full, st);
        default: return dispatch_hop<REP, S, CLOV_NONE>(a, dag, has_a, norm, full, st);
    }
}

template <int REP, typename S>
hipError_t dispatch_rupd(const HopArgs &a, hipStream_t st, int clov)
{
    if constexpr (clover_capable(REP)) {
        if (clov == CLOV_SELF) {
            launch_hop_kernel<REP, S, true, true, true, false, true, CLOV_SELF>(a, st);
            return hipGetLastError();
        }
    }
    launch_hop_kernel<REP, S, true, true, true, false, true, CLOV_NONE>(a, st);
    return hipGetLastError();
}

}  // namespace

}  // namespace hrd
