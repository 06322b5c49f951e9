// Batched multi-right-hand-side / mixed-volume execution.  The paper advises
// local volumes of at least 16^4 for SU(2) (Sec. 3); small lattices and many
// right-hand sides are gathered here into single persistent launches:
//
// * a tile is (problem, block of sites, group of G right-hand sides); a
//   thread owns one site of the tile, loads each of its 8 links once and
//   applies it to the G spinors of the group, so the gauge field is read once
//   per site for the whole group;
// * one persistent grid per hopping stage covers every problem (mixed
//   volumes and representations): each XCD walks its own contiguous range of
//   tiles, and the tiles of one site block are adjacent, so the links of a
//   site block are re-read from that XCD's L2 by the next group;
// * per-problem geometry comes from a descriptor table in device memory.
//
// The batched CG runs one independent mixed-precision reliable-update CG per
// right-hand side (FP32 operator stages batched, per-RHS FP64 scalars and
// reductions, FP64 residual recomputation), masking converged systems.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_util.h"
#include "hop.h"

namespace hrd {

namespace {

constexpr int kMaxProb = 64;
constexpr int kMaxRhs = 64;
// buffer slots of a problem: operator stages use 0..4; the batched CG keeps
// its ring of search directions in slots kBufRing .. kBufRing + kPRing - 1
constexpr int kBufRing = 4;
constexpr int kNumBuf = kBufRing + kPRing;
constexpr int kVecBlocks = 64;  // x-blocks per right-hand side in vector kernels

struct BatchDesc {
    Geom g;
    int rep;
    int nrhs;
    int rhs_base;   // global index of the problem's first right-hand side
    int tile_base;  // first tile of this problem
    int ntiles;
    int nsb;        // site blocks
    int ngroups;    // right-hand-side groups
    double m;       // 4 + m0
    const void *U32;
    size_t fbytes;  // bytes of one FP32 half field
    char *buf[kNumBuf];
};

// Per right-hand side view for the vector stages of the batched CG: p32 is
// the right-hand side's field in ring slot 0, slot s at p32 + s * pslot.
struct RhsDesc {
    int Vh, ncomp, nsb, pad;
    size_t n16;    // 16-byte elements of one FP32 half field
    size_t pslot;  // bytes between ring slots
    char *x64, *r32, *p32;
};

enum BatchMode { M_NORMAL = 0, M_RELIABLE = 1, M_DONE = 2 };

// One direction of the stencil for one right-hand side, with the link
// already in registers: project the neighbour spinor, apply the boundary sign,
// multiply by U (forward) or U^+ (backward), reconstruct and accumulate.
template <int MU, int SIG, bool BWD, int REP>
__device__ __forceinline__ void dir_term(const typename LinkIO<REP, float>::Link &l, const char *src, int Vh, int j,
                                         bool neg, Cx<float> (&acc)[4 * NCol<REP>::value])
{
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    Cx<float> psi[NC];
    SpinorIO<float>::template load<NC>(src, Vh, j, psi);
    Cx<float> h0[N], h1[N], u0[N], u1[N];
    project<MU, SIG, N, float>(psi, h0, h1);
    if (neg) {
#pragma unroll
        for (int c = 0; c < N; c++) {
            h0[c] = -h0[c];
            h1[c] = -h1[c];
        }
    }
    if constexpr (BWD) {
        link_mul_dag(l, h0, u0);
        link_mul_dag(l, h1, u1);
    } else {
        link_mul(l, h0, u0);
        link_mul(l, h1, u1);
    }
    reconstruct<MU, SIG, N, float>(acc, u0, u1);
}

// Block-wide sum of ||out||^2 for one right-hand side of a tile; every
// thread of the block reaches it.
__device__ __forceinline__ void tile_norm_partial(double nrm, double *dst)
{
    __shared__ double part[16];
    for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); wv++) t += part[wv];
        *dst = t;
    }
    __syncthreads();
}

// A tile of a dense SU(N > 2) format: N x N links do not fit in registers,
// so each right-hand side streams them by row (from L2 after the first
// right-hand side of the tile) through the single-problem direction terms:
// the same operations in the same order as the single-problem kernel.
template <int REP, bool DAG, bool EPI2, bool RUPD>
__device__ __forceinline__ void batched_tile_dense(const BatchDesc &d, int sb, int r0, int gcount, int w, bool in,
                                                   int parity, int src_id, int self_id, int dst_id, const int *mode,
                                                   double *partials, int part_stride, const double *sc)
{
    constexpr int NC = 4 * NCol<REP>::value;
    const Geom &g = d.g;
    int idx = 0;
    Site s{};
    if (in) s = slab_site(g, w, parity, &idx);
    const float ca = (float)d.m, cb = EPI2 ? (float)(0.5 / d.m) : -0.5f;
#pragma unroll 1
    for (int k = 0; k < gcount; k++) {
        const int rhs = r0 + k;
        if (mode && mode[d.rhs_base + rhs] == M_DONE) continue;  // uniform
        double nrm = 0;
        if (in) {
            const char *src = d.buf[src_id] + (size_t)rhs * d.fbytes;
            Cx<float> acc[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) acc[c] = Cx<float>{0.f, 0.f};
            hop_dir_dense<0, DAG, REP, float>(g, s, idx, parity, d.U32, src, acc);
            hop_dir_dense<1, DAG, REP, float>(g, s, idx, parity, d.U32, src, acc);
            hop_dir_dense<2, DAG, REP, float>(g, s, idx, parity, d.U32, src, acc);
            hop_dir_dense<3, DAG, REP, float>(g, s, idx, parity, d.U32, src, acc);
            Cx<float> out[NC];
            if constexpr (EPI2) {
                Cx<float> sv[NC];
                SpinorIO<float>::template load<NC>(d.buf[self_id] + (size_t)rhs * d.fbytes, g.Vh, idx, sv);
#pragma unroll
                for (int c = 0; c < NC; c++) out[c] = axpby(ca, sv[c], cb, acc[c]);
                if constexpr (RUPD) {
                    const float alpha = (float)sc[(size_t)(d.rhs_base + rhs) * S_COUNT + S_ALPHA];
                    Cx<float> rv[NC];
                    SpinorIO<float>::template load<NC>(d.buf[dst_id] + (size_t)rhs * d.fbytes, g.Vh, idx, rv);
#pragma unroll
                    for (int c = 0; c < NC; c++) out[c] = Cx<float>{rv[c].re - alpha * out[c].re,
                                                                    rv[c].im - alpha * out[c].im};
                }
#pragma unroll
                for (int c = 0; c < NC; c++) nrm += (double)out[c].re * out[c].re + (double)out[c].im * out[c].im;
            } else {
#pragma unroll
                for (int c = 0; c < NC; c++) out[c] = cb * acc[c];
            }
            SpinorIO<float>::template store<NC, !RUPD>(d.buf[dst_id] + (size_t)rhs * d.fbytes, g.Vh, idx, out);
        }
        if (EPI2 && partials != nullptr) tile_norm_partial(nrm, &partials[(size_t)(d.rhs_base + rhs) * part_stride + sb]);
    }
}

// One tile: sites [sb * blockDim, +blockDim) of the target parity, right-hand
// sides [grp * G, +G) of the problem.  Each thread loads its site's 8 links
// once into registers and then applies them to the right-hand sides one
// after another (each with all 8 neighbour loads in flight), so the
// register footprint does not grow with G.  EPI2: out = m self + acc / (2m),
// plus per-right-hand-side ||out||^2 partials when `partials` is not NULL;
// else out = -acc / 2.  RUPD (with EPI2, batched CG): dst is the residual r,
// updated as r -= alpha out with the right-hand side's alpha from sc, and the
// partials are those of ||r||^2.
template <int REP, bool DAG, bool EPI2, bool RUPD>
__device__ __forceinline__ void batched_tile(const BatchDesc &d, int sb, int grp, int G, int parity, int src_id,
                                             int self_id, int dst_id, const int *mode, double *partials,
                                             int part_stride, const double *sc)
{
    constexpr int NC = 4 * NCol<REP>::value;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    using LIO = LinkIO<REP, float>;
    const Geom &g = d.g;
    const int r0 = grp * G;
    const int gcount = min(G, d.nrhs - r0);  // >= 1: groups start below nrhs
    bool any = false;
    for (int k = 0; k < gcount; k++) any = any || !mode || mode[d.rhs_base + r0 + k] != M_DONE;
    if (!any) return;  // uniform across the block
    const int w = sb * (int)blockDim.x + (int)threadIdx.x;
    const bool in = w < g.Vh;
    if constexpr (is_dense(REP)) {
        batched_tile_dense<REP, DAG, EPI2, RUPD>(d, sb, r0, gcount, w, in, parity, src_id, self_id, dst_id, mode,
                                                 partials, part_stride, sc);
        return;
    }
    int idx = 0;
    int jf[4] = {0, 0, 0, 0}, jb[4] = {0, 0, 0, 0};
    bool nf = false, nb = false;
    typename LIO::Link lf[4], lb[4];
    if (in) {
        const Site s = slab_site(g, w, parity, &idx);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            jf[mu] = nbr_fwd(g, s, mu);
            jb[mu] = nbr_bwd(g, s, mu);
            lf[mu] = LIO::template load<true>(d.U32, g.Vh, parity, mu, idx);
            lb[mu] = LIO::template load<true>(d.U32, g.Vh, 1 - parity, mu, jb[mu]);
        }
        nf = s.x[0] == g.L[0] - 1;
        nb = s.x[0] == 0;
    }
    const float ca = (float)d.m, cb = EPI2 ? (float)(0.5 / d.m) : -0.5f;
#pragma unroll 1
    for (int k = 0; k < gcount; k++) {
        const int rhs = r0 + k;
        if (mode && mode[d.rhs_base + rhs] == M_DONE) continue;  // uniform
        double nrm = 0;
        if (in) {
            const char *src = d.buf[src_id] + (size_t)rhs * d.fbytes;
            Cx<float> acc[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) acc[c] = Cx<float>{0.f, 0.f};
            dir_term<0, SF, false, REP>(lf[0], src, g.Vh, jf[0], nf, acc);
            dir_term<0, SB, true, REP>(lb[0], src, g.Vh, jb[0], nb, acc);
            dir_term<1, SF, false, REP>(lf[1], src, g.Vh, jf[1], false, acc);
            dir_term<1, SB, true, REP>(lb[1], src, g.Vh, jb[1], false, acc);
            dir_term<2, SF, false, REP>(lf[2], src, g.Vh, jf[2], false, acc);
            dir_term<2, SB, true, REP>(lb[2], src, g.Vh, jb[2], false, acc);
            dir_term<3, SF, false, REP>(lf[3], src, g.Vh, jf[3], false, acc);
            dir_term<3, SB, true, REP>(lb[3], src, g.Vh, jb[3], false, acc);
            Cx<float> out[NC];
            if constexpr (EPI2) {
                Cx<float> sv[NC];
                SpinorIO<float>::template load<NC>(d.buf[self_id] + (size_t)rhs * d.fbytes, g.Vh, idx, sv);
#pragma unroll
                for (int c = 0; c < NC; c++) out[c] = axpby(ca, sv[c], cb, acc[c]);
                if constexpr (RUPD) {
                    const float alpha = (float)sc[(size_t)(d.rhs_base + rhs) * S_COUNT + S_ALPHA];
                    Cx<float> rv[NC];
                    SpinorIO<float>::template load<NC>(d.buf[dst_id] + (size_t)rhs * d.fbytes, g.Vh, idx, rv);
#pragma unroll
                    for (int c = 0; c < NC; c++) out[c] = Cx<float>{rv[c].re - alpha * out[c].re,
                                                                    rv[c].im - alpha * out[c].im};
                }
#pragma unroll
                for (int c = 0; c < NC; c++) nrm += (double)out[c].re * out[c].re + (double)out[c].im * out[c].im;
            } else {
#pragma unroll
                for (int c = 0; c < NC; c++) out[c] = cb * acc[c];
            }
            SpinorIO<float>::template store<NC, !RUPD>(d.buf[dst_id] + (size_t)rhs * d.fbytes, g.Vh, idx, out);
        }
        // block-wide sum of ||out||^2, only when the caller wants it (a
        // uniform kernel argument)
        if (EPI2 && partials != nullptr) tile_norm_partial(nrm, &partials[(size_t)(d.rhs_base + rhs) * part_stride + sb]);
    }
}

// GROUP 0: problems in the SU(2) formats, in any mix; otherwise every
// problem uses the dense SU(N > 2) format GROUP.
template <bool DAG, bool EPI2, bool RUPD, int GROUP>
__global__ __launch_bounds__(256) void batched_hop_kernel(const BatchDesc *descs, int nprob, int ntiles, int G,
                                                          int parity, int src_id, int self_id, int dst_id,
                                                          const int *mode, double *partials, int part_stride,
                                                          const double *sc)
{
    // each XCD walks its own contiguous range of tiles (gridDim.x is a multiple of 8)
    const int xcd = blockIdx.x % kNumXcd;
    const int slot = blockIdx.x / kNumXcd;
    const int per = gridDim.x / kNumXcd;
    const int t0 = (int)((long)ntiles * xcd / kNumXcd);
    const int t1 = (int)((long)ntiles * (xcd + 1) / kNumXcd);
    int p = 0;
    for (int tile = t0 + slot; tile < t1; tile += per) {
        while (p + 1 < nprob && tile >= descs[p + 1].tile_base) p++;
        while (tile < descs[p].tile_base) p--;
        const BatchDesc &d = descs[p];
        const int local = tile - d.tile_base;
        const int sb = local / d.ngroups;
        const int grp = local - sb * d.ngroups;
        if constexpr (GROUP != 0) {
            batched_tile<GROUP, DAG, EPI2, RUPD>(d, sb, grp, G, parity, src_id, self_id, dst_id, mode, partials,
                                                 part_stride, sc);
            continue;
        }
        switch (d.rep) {
            case HRD_FUND:
                batched_tile<HRD_FUND, DAG, EPI2, RUPD>(d, sb, grp, G, parity, src_id, self_id, dst_id, mode,
                                                  partials, part_stride, sc);
                break;
            case HRD_ADJ:
                batched_tile<HRD_ADJ, DAG, EPI2, RUPD>(d, sb, grp, G, parity, src_id, self_id, dst_id, mode,
                                                 partials, part_stride, sc);
                break;
            case HRD_FUND_SU2:
                batched_tile<HRD_FUND_SU2, DAG, EPI2, RUPD>(d, sb, grp, G, parity, src_id, self_id, dst_id, mode,
                                                      partials, part_stride, sc);
                break;
            default:
                batched_tile<HRD_ADJ_SU2, DAG, EPI2, RUPD>(d, sb, grp, G, parity, src_id, self_id, dst_id, mode,
                                                     partials, part_stride, sc);
                break;
        }
    }
}

// ----- per right-hand-side vector stages of the batched CG -----------------

__device__ __forceinline__ double blk_sum256(double v)
{
    __shared__ double part[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) s = part[0] + part[1] + part[2] + part[3];
    __syncthreads();
    return s;
}

// Ring of FP32 search directions shared in lockstep by all right-hand sides
// (grid: kVecBlocks x nrhs, thread per (F32 plane q, site j), F64 planes 2q,
// 2q+1).  For right-hand side r, unless done: when `flush_all` is set or r is
// in a reliable update, x64 += alpha_s f64(p_s) over its pending slots
// s = lo[r] .. j in order (alpha_s = ahist[r * kPRing + s]); when r is normal
// and dst >= 0, p_dst = r32 + beta p_j.
__global__ __launch_bounds__(256) void bcg_ring_kernel(const RhsDesc *rd, const int *mode, const int *lo,
                                                       const double *sc, const double *ahist, int j, int dst,
                                                       int flush_all)
{
    const int r = blockIdx.y;
    const int md = mode[r];
    if (md == M_DONE) return;
    const bool flush = flush_all || md == M_RELIABLE;
    const bool adv = md == M_NORMAL && dst >= 0;
    if (!flush && !adv) return;
    const RhsDesc d = rd[r];
    const int s0 = lo[r];
    const double *al = ahist + (size_t)r * kPRing;
    const float beta = (float)sc[r * S_COUNT + S_BETA];
    const int npl = d.ncomp / 2;
    const long n = (long)npl * d.Vh;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
        const MixOff o = mix_off(t, d.Vh, npl);
        if (flush) {
            double2 *X0 = reinterpret_cast<double2 *>(d.x64 + o.f64a);
            double2 *X1 = reinterpret_cast<double2 *>(d.x64 + o.f64b);
            double2 x0 = *X0, x1 = *X1;
            for (int sl = s0; sl <= j; sl++) {
                const double alpha = al[sl];
                const float4 pv = *reinterpret_cast<const float4 *>(d.p32 + (size_t)sl * d.pslot + o.f32);
                x0.x += alpha * (double)pv.x;
                x0.y += alpha * (double)pv.y;
                x1.x += alpha * (double)pv.z;
                x1.y += alpha * (double)pv.w;
            }
            *X0 = x0;
            *X1 = x1;
        }
        if (adv) {
            const float4 pv = *reinterpret_cast<const float4 *>(d.p32 + (size_t)j * d.pslot + o.f32);
            const float4 rv = *reinterpret_cast<const float4 *>(d.r32 + o.f32);
            *reinterpret_cast<float4 *>(d.p32 + (size_t)dst * d.pslot + o.f32) =
                make_float4(rv.x + beta * pv.x, rv.y + beta * pv.y, rv.z + beta * pv.z, rv.w + beta * pv.w);
        }
    }
}

// Per right-hand side: alpha = rr / pAp from the hop partials (count nsb),
// also kept in ring slot j of ahist.
__global__ __launch_bounds__(256) void bcg_alpha_kernel(const RhsDesc *rd, const int *mode, const double *partials,
                                                        int part_stride, double *sc, double *ahist, int j)
{
    const int r = blockIdx.x;
    if (mode[r] == M_DONE) return;
    const int n = rd[r].nsb;
    double s = 0;
    for (int k = threadIdx.x; k < n; k += 256) s += partials[(size_t)r * part_stride + k];
    s = blk_sum256(s);
    if (threadIdx.x == 0) {
        double *c = sc + r * S_COUNT;
        c[S_PAP] = s;
        double alpha = 0.0;
        if (!(s > 0.0) || !isfinite(s)) c[S_FLAG] = 1.0;
        else alpha = c[S_RR] / s;
        c[S_ALPHA] = alpha;
        ahist[(size_t)r * kPRing + j] = alpha;
    }
}

// Per right-hand side: rr_new from the partials of the residual-updating
// stage (count nsb), beta = rr_new / rr.
__global__ __launch_bounds__(256) void bcg_beta_kernel(const RhsDesc *rd, const int *mode, const double *partials,
                                                       int part_stride, double *sc)
{
    const int r = blockIdx.x;
    if (mode[r] == M_DONE) return;
    const int n = rd[r].nsb;
    double s = 0;
    for (int k = threadIdx.x; k < n; k += 256) s += partials[(size_t)r * part_stride + k];
    s = blk_sum256(s);
    if (threadIdx.x == 0) {
        double *c = sc + r * S_COUNT;
        c[S_RRNEW] = s;
        if (!isfinite(s)) {
            c[S_FLAG] = 2.0;
            c[S_BETA] = 0.0;
        } else {
            c[S_BETA] = c[S_RR] > 0.0 ? s / c[S_RR] : 0.0;
        }
        c[S_RROLD] = c[S_RR];
        c[S_RR] = s;
    }
}

// ----- host side ------------------------------------------------------------

struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    void *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += n;
        return p;
    }
    size_t used() const { return (off + 255) & ~(size_t)255; }
};

// Kernel family of a batch: 0 for the SU(2) formats (mixed freely), else the
// dense SU(N > 2) format every problem of the batch uses.
int batch_group(int rep) { return is_dense(rep) ? rep : 0; }

hrd_status check_problems(const hrd_problem *probs, int nprob, bool need_u64)
{
    if (!probs || nprob < 1 || nprob > kMaxProb) return fail(HRD_EINVAL, "nprob must be in 1..%d", kMaxProb);
    int total = 0;
    for (int i = 0; i < nprob; i++) {
        const hrd_problem &p = probs[i];
        HRD_TRY(check_lattice(&p.lat));
        HRD_TRY(check_rep_prec(p.rep, HRD_F32));
        if (is_dense(p.rep) ? p.rep != probs[0].rep : is_dense(probs[0].rep))
            return fail(HRD_EINVAL, "problem %d: a batch takes the SU(2) formats in any mix, or problems of one dense "
                                    "SU(N) format", i);
        if (p.nrhs < 1 || p.nrhs > kMaxRhs) return fail(HRD_EINVAL, "problem %d: nrhs must be in 1..%d", i, kMaxRhs);
        if (!p.U32 || !p.src || !p.dst) return fail(HRD_EINVAL, "problem %d: NULL pointer", i);
        if (need_u64 && !p.U64) return fail(HRD_EINVAL, "problem %d: the batched CG needs U64", i);
        if (!std::isfinite(p.m0) || 4.0 + p.m0 == 0.0) return fail(HRD_EINVAL, "problem %d: invalid m0", i);
        total += p.nrhs;
    }
    if (total > kMaxProb * 4) return fail(HRD_EINVAL, "too many right-hand sides in total (%d)", total);
    return HRD_OK;
}

hrd_tune resolve_tune(const hrd_tune *t)
{
    hrd_tune r{128, 4, 128, 4, 0};
    if (t) {
        if (t->sites_per_tile > 0) r.sites_per_tile = t->sites_per_tile;
        if (t->rhs_per_tile > 0) r.rhs_per_tile = t->rhs_per_tile;
        if (t->block_threads > 0) r.block_threads = t->block_threads;
        if (t->blocks_per_cu > 0) r.blocks_per_cu = t->blocks_per_cu;
        if (t->slab_width > 0) r.slab_width = t->slab_width;
    }
    r.block_threads = r.sites_per_tile;  // one thread per site of a tile
    return r;
}

hrd_status check_tune(const hrd_tune &t)
{
    if (t.sites_per_tile != 64 && t.sites_per_tile != 128 && t.sites_per_tile != 256)
        return fail(HRD_EINVAL, "sites_per_tile must be 64, 128 or 256");
    if (t.rhs_per_tile < 1 || t.rhs_per_tile > kMaxRhs) return fail(HRD_EINVAL, "rhs_per_tile must be in 1..%d", kMaxRhs);
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16) return fail(HRD_EINVAL, "blocks_per_cu must be in 1..16");
    if (t.slab_width < 0) return fail(HRD_EINVAL, "slab_width must be >= 0");
    return HRD_OK;
}

// x1-slab width of a problem's traversal: the requested width rounded down to
// a divisor of L1, or, when 0, the widest slab whose t-slice holds at most
// 6912 sites counting each of the G right-hand sides swept together (the same
// budget as the single-right-hand-side operator).
int batched_slab(const int dims[4], int G, int requested)
{
    int best = 1;
    if (requested > 0) {
        for (int b = 1; b <= dims[1] && b <= requested; b++)
            if (dims[1] % b == 0) best = b;
        return best;
    }
    const long R = (long)dims[2] * dims[3] / 2;
    for (int b = 1; b <= dims[1]; b++)
        if (dims[1] % b == 0 && (long)b * R * G <= 6912) best = b;
    return best;
}

// Fill the descriptor table; returns total tiles.
int build_descs(const hrd_problem *probs, int nprob, const hrd_tune &t, std::vector<BatchDesc> &d, int *max_nsb)
{
    d.assign(nprob, BatchDesc{});
    int tiles = 0, rhs = 0;
    *max_nsb = 0;
    for (int i = 0; i < nprob; i++) {
        BatchDesc &b = d[i];
        b.g = make_geom(probs[i].lat.dims, batched_slab(probs[i].lat.dims, t.rhs_per_tile, t.slab_width));
        b.rep = probs[i].rep;
        b.nrhs = probs[i].nrhs;
        b.rhs_base = rhs;
        b.nsb = (b.g.Vh + t.sites_per_tile - 1) / t.sites_per_tile;
        b.ngroups = (b.nrhs + t.rhs_per_tile - 1) / t.rhs_per_tile;
        b.ntiles = b.nsb * b.ngroups;
        b.tile_base = tiles;
        b.m = 4.0 + probs[i].m0;
        b.U32 = probs[i].U32;
        b.fbytes = spinor_bytes(&probs[i].lat, b.rep, HRD_F32, 1);
        tiles += b.ntiles;
        rhs += b.nrhs;
        *max_nsb = std::max(*max_nsb, b.nsb);
    }
    return tiles;
}

template <bool DAG, bool EPI2, bool RUPD>
hipError_t launch_stage_t(const hrd_tune &t, hipStream_t st, const BatchDesc *dd, int nprob, int ntiles, int parity,
                          int s, int self, int dst, const int *mode, double *parts, int ps, const double *sc,
                          int group)
{
    int grid = kNumCu * t.blocks_per_cu;
    grid = (grid / kNumXcd) * kNumXcd;
#define HRD_BATCHED(GRP)                                                                                        \
    hipLaunchKernelGGL((batched_hop_kernel<DAG, EPI2, RUPD, GRP>), dim3(grid), dim3(t.sites_per_tile), 0, st, dd, \
                       nprob, ntiles, t.rhs_per_tile, parity, s, self, dst, mode, parts, ps, sc)
    switch (group) {
        case 0: HRD_BATCHED(0); break;
        case HRD_CPLX3: HRD_BATCHED(HRD_CPLX3); break;
        case HRD_CPLX4: HRD_BATCHED(HRD_CPLX4); break;
        case HRD_CPLX6: HRD_BATCHED(HRD_CPLX6); break;
        case HRD_REAL8: HRD_BATCHED(HRD_REAL8); break;
        case HRD_SU3_ROW2: HRD_BATCHED(HRD_SU3_ROW2); break;
        case HRD_CPLX10: HRD_BATCHED(HRD_CPLX10); break;
        default: HRD_BATCHED(HRD_REAL15); break;
    }
#undef HRD_BATCHED
    return hipGetLastError();
}

// One hopping stage over every problem.  sc != NULL (batched CG, with epi2
// and dagger): the stage updates the residual in buffer dst (r -= alpha Ap).
hipError_t launch_stage(int group, const hrd_tune &t, bool dag, bool epi2, hipStream_t st, const BatchDesc *dd,
                        int nprob, int ntiles, int parity, int s, int self, int dst, const int *mode, double *parts,
                        int ps, const double *sc = nullptr)
{
    if (sc) {
        if (!dag || !epi2) return hipErrorInvalidValue;
        return launch_stage_t<true, true, true>(t, st, dd, nprob, ntiles, parity, s, self, dst, mode, parts, ps, sc, group);
    }
    if (dag) {
        if (epi2) return launch_stage_t<true, true, false>(t, st, dd, nprob, ntiles, parity, s, self, dst, mode, parts, ps, sc, group);
        return launch_stage_t<true, false, false>(t, st, dd, nprob, ntiles, parity, s, self, dst, mode, parts, ps, sc, group);
    }
    if (epi2) return launch_stage_t<false, true, false>(t, st, dd, nprob, ntiles, parity, s, self, dst, mode, parts, ps, sc, group);
    return launch_stage_t<false, false, false>(t, st, dd, nprob, ntiles, parity, s, self, dst, mode, parts, ps, sc, group);
}

// Workspace of the batched apply: descriptor table, then one FP32 odd
// temporary per right-hand side (HRD_EO).
size_t apply_ws(const hrd_problem *probs, int nprob, hrd_parity parity, BatchDesc **dd, char ***tmp, void *work)
{
    Carve c(work);
    *dd = (BatchDesc *)c.take(sizeof(BatchDesc) * kMaxProb);
    static thread_local char *tmps[kMaxProb];
    for (int i = 0; i < nprob; i++) {
        const size_t fb = spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F32, 1);
        tmps[i] = parity == HRD_EO ? (char *)c.take(fb * probs[i].nrhs) : nullptr;
    }
    if (tmp) *tmp = tmps;
    return c.used();
}

// Runs the batched hopping stages of `parity` over the prepared table.
hrd_status run_batched(const std::vector<BatchDesc> &hd, BatchDesc *dd, int ntiles, const hrd_tune &t,
                       hrd_parity parity, bool dag, hipStream_t st)
{
    const int np = (int)hd.size();
    const int grp = batch_group(hd[0].rep);
    HRD_TRY(check_hip(hipMemcpyAsync(dd, hd.data(), sizeof(BatchDesc) * np, hipMemcpyHostToDevice, st), "desc upload"));
    hipError_t e;
    if (parity == HRD_EO) {
        // buffers: 0 src, 1 dst, 2 tmp
        e = launch_stage(grp, t, dag, false, st, dd, np, ntiles, 1, 0, 0, 2, nullptr, nullptr, 0);
        if (e == hipSuccess) e = launch_stage(grp, t, dag, true, st, dd, np, ntiles, 0, 2, 0, 1, nullptr, nullptr, 0);
    } else {
        const int target = parity == HRD_HOP_EO ? 0 : 1;
        e = launch_stage(grp, t, dag, false, st, dd, np, ntiles, target, 0, 0, 1, nullptr, nullptr, 0);
    }
    return check_hip(e, "batched hop launch");
}

}  // namespace

}  // namespace hrd

using namespace hrd;

extern "C" {

size_t hrd_batched_workspace_bytes(const hrd_problem *probs, int nprob, hrd_parity parity)
{
    if (check_problems(probs, nprob, false) != HRD_OK) return 0;
    BatchDesc *dd;
    return apply_ws(probs, nprob, parity, &dd, nullptr, nullptr);
}

hrd_status hrd_dirac_apply_batched(const hrd_problem *probs, int nprob, hrd_parity parity, int dagger,
                                   const hrd_tune *tune, void *work, size_t work_bytes, void *stream)
{
    HRD_TRY(check_problems(probs, nprob, false));
    if (parity != HRD_EO && parity != HRD_HOP_EO && parity != HRD_HOP_OE)
        return fail(HRD_EINVAL, "batched parity must be HRD_EO, HRD_HOP_EO or HRD_HOP_OE");
    const hrd_tune t = resolve_tune(tune);
    HRD_TRY(check_tune(t));
    if (!work) return fail(HRD_EINVAL, "NULL workspace");
    BatchDesc *dd;
    char **tmps;
    const size_t need = apply_ws(probs, nprob, parity, &dd, &tmps, work);
    if (work_bytes < need) return fail(HRD_ESIZE, "workspace %zu < %zu bytes", work_bytes, need);
    for (int i = 0; i < nprob; i++) {
        const size_t fb = spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F32, 1) * probs[i].nrhs;
        for (int j = 0; j < nprob; j++) {
            const size_t fbj = spinor_bytes(&probs[j].lat, probs[j].rep, HRD_F32, 1) * probs[j].nrhs;
            if (overlap(probs[i].dst, fb, probs[j].src, fbj)) return fail(HRD_EALIAS, "problem %d dst overlaps a source", i);
            if (j != i && overlap(probs[i].dst, fb, probs[j].dst, fbj)) return fail(HRD_EALIAS, "destinations overlap");
        }
        if (overlap(work, need, probs[i].dst, fb) || overlap(work, need, probs[i].src, fb))
            return fail(HRD_EALIAS, "workspace overlaps problem %d", i);
    }
    std::vector<BatchDesc> hd;
    int max_nsb;
    const int ntiles = build_descs(probs, nprob, t, hd, &max_nsb);
    for (int i = 0; i < nprob; i++) {
        hd[i].buf[0] = (char *)probs[i].src;
        hd[i].buf[1] = (char *)probs[i].dst;
        hd[i].buf[2] = tmps[i];
    }
    return run_batched(hd, dd, ntiles, t, parity, dagger != 0, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched mixed-precision CG
// ---------------------------------------------------------------------------

namespace hrd {
namespace {

struct BcgWork {
    BatchDesc *dd;
    RhsDesc *rd;
    int *mode;
    double *sc, *parts, *ahist;
    // FP64 temporaries sized for the largest problem (reliable updates)
    void *q64, *Ap64, *t64, *r64;
    // per problem FP32 buffers (nrhs fields each): t (odd), q, r, and the
    // ring of kPRing search-direction slots
    char *f32[kMaxProb][3];
    char *ring[kMaxProb];
};

size_t bcg_carve(const hrd_problem *probs, int nprob, void *work, BcgWork *w)
{
    Carve c(work);
    BcgWork t{};
    int total = 0;
    size_t max64 = 0;
    int max_nsb = 0;
    for (int i = 0; i < nprob; i++) {
        total += probs[i].nrhs;
        max64 = std::max(max64, spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F64, 1));
        const Geom g = make_geom(probs[i].lat.dims);
        max_nsb = std::max(max_nsb, (g.Vh + 63) / 64);
    }
    t.dd = (BatchDesc *)c.take(sizeof(BatchDesc) * kMaxProb);
    t.rd = (RhsDesc *)c.take(sizeof(RhsDesc) * total);
    t.mode = (int *)c.take(sizeof(int) * 2 * total);  // modes, then first pending ring slots
    t.sc = (double *)c.take(sizeof(double) * S_COUNT * total);
    t.parts = (double *)c.take(sizeof(double) * (size_t)std::max(max_nsb, kRedBlocks) * total);
    t.ahist = (double *)c.take(sizeof(double) * kPRing * total);
    t.q64 = c.take(max64);
    t.Ap64 = c.take(max64);
    t.t64 = c.take(max64);
    t.r64 = c.take(max64);
    for (int i = 0; i < nprob; i++) {
        const size_t fb = spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F32, 1) * probs[i].nrhs;
        for (int k = 0; k < 3; k++) t.f32[i][k] = (char *)c.take(fb);
        t.ring[i] = (char *)c.take(fb * kPRing);
    }
    if (w) *w = t;
    return c.used();
}

}  // namespace
}  // namespace hrd

extern "C" {

size_t hrd_cg_batched_workspace_bytes(const hrd_problem *probs, int nprob)
{
    if (check_problems(probs, nprob, true) != HRD_OK) return 0;
    return bcg_carve(probs, nprob, nullptr, nullptr);
}

hrd_status hrd_cg_solve_batched(const hrd_problem *probs, int nprob, double tol, int maxiter, double delta,
                                const hrd_tune *tune, void *work, size_t work_bytes, hrd_cg_info *infos, void *stream)
{
    const auto t_start = std::chrono::steady_clock::now();
    HRD_TRY(check_problems(probs, nprob, true));
    const int grp = batch_group(probs[0].rep);
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(HRD_EINVAL, "tol must be positive");
    if (maxiter < 0) return fail(HRD_EINVAL, "maxiter must be >= 0");
    if (!work) return fail(HRD_EINVAL, "NULL workspace");
    hrd_tune t = resolve_tune(tune);
    HRD_TRY(check_tune(t));
    if (delta <= 0.0) delta = kDeltaMixed;
    const size_t need = bcg_carve(probs, nprob, nullptr, nullptr);
    if (work_bytes < need) return fail(HRD_ESIZE, "workspace %zu < %zu bytes", work_bytes, need);
    for (int i = 0; i < nprob; i++) {
        const size_t fb = spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F64, 1) * probs[i].nrhs;
        if (overlap(probs[i].dst, fb, probs[i].src, fb)) return fail(HRD_EALIAS, "problem %d: x overlaps b", i);
        if (overlap(work, need, probs[i].dst, fb) || overlap(work, need, probs[i].src, fb))
            return fail(HRD_EALIAS, "workspace overlaps problem %d", i);
    }
    const hipStream_t st = (hipStream_t)stream;
    BcgWork w;
    bcg_carve(probs, nprob, work, &w);

    std::vector<BatchDesc> hd;
    int max_nsb;
    const int ntiles = build_descs(probs, nprob, t, hd, &max_nsb);
    const int part_stride = std::max(max_nsb, kRedBlocks);
    for (int i = 0; i < nprob; i++) {
        for (int k = 0; k < 3; k++) hd[i].buf[k] = w.f32[i][k];
        for (int sl = 0; sl < kPRing; sl++) hd[i].buf[kBufRing + sl] = w.ring[i] + (size_t)sl * hd[i].nrhs * hd[i].fbytes;
    }
    enum { B_T = 0, B_Q = 1, B_R = 2 };
    int total = 0;
    for (int i = 0; i < nprob; i++) total += probs[i].nrhs;
    std::vector<RhsDesc> rdh(total);
    std::vector<int> prob_of(total), slot_of(total);
    for (int i = 0, r = 0; i < nprob; i++)
        for (int k = 0; k < probs[i].nrhs; k++, r++) {
            const Geom &g = hd[i].g;
            RhsDesc &d = rdh[r];
            d.Vh = g.Vh;
            d.ncomp = ncomp_of(probs[i].rep);
            d.nsb = hd[i].nsb;
            d.n16 = hd[i].fbytes / 16;
            d.x64 = (char *)probs[i].dst + (size_t)k * spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F64, 1);
            d.r32 = w.f32[i][B_R] + (size_t)k * hd[i].fbytes;
            d.p32 = w.ring[i] + (size_t)k * hd[i].fbytes;
            d.pslot = (size_t)hd[i].nrhs * hd[i].fbytes;
            prob_of[r] = i;
            slot_of[r] = k;
        }
    // mode of each right-hand side, then its first ring slot whose update is
    // not yet in x (uploaded together)
    std::vector<int> ml(2 * (size_t)total, 0);
    int *mode = ml.data();
    int *lo = ml.data() + total;
    std::vector<double> sc((size_t)S_COUNT * total);
    std::vector<double> bnorm(total), rmax(total), dlt(total, delta);
    std::vector<hrd_cg_info> inf(total);
    std::vector<hrd_status> stat(total, HRD_OK);

#define BT(expr, what) HRD_TRY(check_hip((expr), what))
    BT(hipMemcpyAsync(w.dd, hd.data(), sizeof(BatchDesc) * nprob, hipMemcpyHostToDevice, st), "desc upload");
    BT(hipMemcpyAsync(w.rd, rdh.data(), sizeof(RhsDesc) * total, hipMemcpyHostToDevice, st), "rhs upload");
    BT(launch_zero(sizeof(double) * S_COUNT * total, w.sc, st), "zero");

    auto b64_of = [&](int r) {
        const int i = prob_of[r];
        return (const char *)probs[i].src + (size_t)slot_of[r] * spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F64, 1);
    };
    // FP64 residual of one right-hand side: r64 = b - A x ; r32 = f32(r64) ; sc[S_RR] = ||r64||^2
    auto residual = [&](int r) -> hrd_status {
        const int i = prob_of[r];
        const Geom &g = hd[i].g;
        const int rep = probs[i].rep;
        const double m0 = probs[i].m0;
        hipError_t e = apply_dhat(rep, HRD_F64, g, probs[i].U64, rdh[r].x64, w.q64, w.t64, m0, false, nullptr, st);
        if (e == hipSuccess) e = apply_dhat(rep, HRD_F64, g, probs[i].U64, w.q64, w.Ap64, w.t64, m0, true, nullptr, st);
        if (e == hipSuccess)
            e = launch_cg_residual_mixed(g.Vh, ncomp_of(rep), b64_of(r), w.Ap64, w.r64, rdh[r].r32, w.parts, st);
        if (e == hipSuccess) e = launch_finalize(w.parts, kRedBlocks, 1, w.sc + (size_t)r * S_COUNT + S_RR, st);
        return check_hip(e, "batched residual");
    };
    auto read_sc = [&]() -> hrd_status {
        HRD_TRY(check_hip(hipMemcpyAsync(sc.data(), w.sc, sizeof(double) * S_COUNT * total, hipMemcpyDeviceToHost, st),
                          "scalars"));
        return check_hip(hipStreamSynchronize(st), "sync");
    };
    auto upload_mode = [&]() {
        return check_hip(hipMemcpyAsync(w.mode, ml.data(), sizeof(int) * 2 * total, hipMemcpyHostToDevice, st),
                         "mode");
    };

    // ||b||^2 and initial residuals
    for (int r = 0; r < total; r++) {
        const int i = prob_of[r];
        const size_t n16 = spinor_bytes(&probs[i].lat, probs[i].rep, HRD_F64, 1) / 16;
        BT(launch_norm_partials(HRD_F64, n16, b64_of(r), w.parts, st), "norm b");
        BT(launch_finalize(w.parts, kRedBlocks, 1, w.sc + (size_t)r * S_COUNT + S_BB, st), "finalize");
        HRD_TRY(residual(r));
    }
    HRD_TRY(read_sc());
    int active = 0;
    for (int r = 0; r < total; r++) {
        const double bb = sc[(size_t)r * S_COUNT + S_BB];
        const double rr = sc[(size_t)r * S_COUNT + S_RR];
        bnorm[r] = std::sqrt(bb);
        if (!std::isfinite(bb) || !std::isfinite(rr)) {
            stat[r] = HRD_EBREAKDOWN;
            mode[r] = M_DONE;
            continue;
        }
        inf[r].true_rel_residual = bb > 0 ? std::sqrt(rr) / bnorm[r] : 0.0;
        inf[r].iterated_rel_residual = inf[r].true_rel_residual;
        if (bb == 0.0 || std::sqrt(rr) <= tol * bnorm[r]) {
            mode[r] = M_DONE;
            if (bb == 0.0) BT(launch_zero(spinor_bytes(&probs[prob_of[r]].lat, probs[prob_of[r]].rep, HRD_F64, 1),
                                          rdh[r].x64, st), "zero x");
            continue;
        }
        rmax[r] = std::sqrt(rr);
        BT(launch_copy(hd[prob_of[r]].fbytes, rdh[r].r32, rdh[r].p32, st), "p = r");
        active++;
    }
    HRD_TRY(upload_mode());

    const dim3 vgrid(kVecBlocks, total);
    // the right-hand sides step through the ring of search directions in
    // lockstep: slot j holds the current p of every active one
    int j = 0;
    int it = 0;
    while (active > 0 && it < maxiter) {
        it++;
        const int P = kBufRing + j;
        // q = D^ p (norm partials), alpha; r -= alpha D^+ q (norm partials)
        BT(launch_stage(grp, t, false, false, st, w.dd, nprob, ntiles, 1, P, P, B_T, w.mode, nullptr, 0), "hop");
        BT(launch_stage(grp, t, false, true, st, w.dd, nprob, ntiles, 0, B_T, P, B_Q, w.mode, w.parts, part_stride), "hop");
        hipLaunchKernelGGL(bcg_alpha_kernel, dim3(total), dim3(256), 0, st, w.rd, w.mode, w.parts, part_stride, w.sc,
                           w.ahist, j);
        BT(hipGetLastError(), "alpha");
        BT(launch_stage(grp, t, true, false, st, w.dd, nprob, ntiles, 1, B_Q, B_Q, B_T, w.mode, nullptr, 0), "hop");
        BT(launch_stage(grp, t, true, true, st, w.dd, nprob, ntiles, 0, B_T, B_Q, B_R, w.mode, w.parts, part_stride, w.sc),
           "hop, r update");
        hipLaunchKernelGGL(bcg_beta_kernel, dim3(total), dim3(256), 0, st, w.rd, w.mode, w.parts, part_stride, w.sc);
        BT(hipGetLastError(), "beta");
        HRD_TRY(read_sc());
        std::vector<int> reliable;
        for (int r = 0; r < total; r++) {
            if (mode[r] == M_DONE) continue;
            inf[r].iters++;
            const double *c = &sc[(size_t)r * S_COUNT];
            if (c[S_FLAG] != 0.0) {
                stat[r] = HRD_EBREAKDOWN;
                mode[r] = M_DONE;
                active--;
                continue;
            }
            const double rn = std::sqrt(c[S_RR]);
            inf[r].iterated_rel_residual = rn / bnorm[r];
            rmax[r] = std::max(rmax[r], rn);
            if (rn < dlt[r] * rmax[r] || rn <= tol * bnorm[r]) {
                mode[r] = M_RELIABLE;
                reliable.push_back(r);
            }
        }
        // normal: p into the next slot (a full ring is folded into x first);
        // reliable: x brought up to date
        const int nj = j + 1 < kPRing ? j + 1 : 0;
        HRD_TRY(upload_mode());
        hipLaunchKernelGGL(bcg_ring_kernel, vgrid, dim3(256), 0, st, w.rd, w.mode, w.mode + total, w.sc, w.ahist, j,
                           nj, nj == 0 ? 1 : 0);
        BT(hipGetLastError(), "ring");
        if (nj == 0)
            for (int r = 0; r < total; r++) lo[r] = 0;
        if (!reliable.empty()) {
            for (int r : reliable) HRD_TRY(residual(r));
            HRD_TRY(read_sc());
            for (int r : reliable) {
                inf[r].reliable_updates++;
                const double rt = std::sqrt(sc[(size_t)r * S_COUNT + S_RR]);
                inf[r].true_rel_residual = rt / bnorm[r];
                if (!std::isfinite(rt)) {
                    stat[r] = HRD_EBREAKDOWN;
                    mode[r] = M_DONE;
                    active--;
                } else if (rt <= tol * bnorm[r]) {
                    mode[r] = M_DONE;
                    active--;
                } else {
                    mode[r] = M_NORMAL;
                    // drift of the FP32 recurrence beyond the threshold: restart
                    // p from r and raise this right-hand side's threshold
                    const double rn = inf[r].iterated_rel_residual * bnorm[r];
                    int bm = kBetaRatio;
                    if (rt > 2.0 * rn) {
                        inf[r].restarts++;
                        dlt[r] = std::min(0.5, 10.0 * dlt[r]);
                        bm = kBetaZero;
                    }
                    BT(launch_cg_ring(HRD_F32, rdh[r].Vh, rdh[r].ncomp, nullptr, rdh[r].p32, rdh[r].pslot, 0, j, nj,
                                      rdh[r].r32, w.sc + (size_t)r * S_COUNT, nullptr, bm, st),
                       "p");
                    lo[r] = nj;
                    rmax[r] = rt;
                }
            }
            HRD_TRY(upload_mode());
        }
        j = nj;
    }
    // x of every unfinished right-hand side still lacks the updates of its
    // slots lo .. j-1
    if (j > 0) {
        HRD_TRY(upload_mode());
        hipLaunchKernelGGL(bcg_ring_kernel, vgrid, dim3(256), 0, st, w.rd, w.mode, w.mode + total, w.sc, w.ahist,
                           j - 1, -1, 1);
        BT(hipGetLastError(), "ring flush");
    }
    hrd_status result = HRD_OK;
    for (int r = 0; r < total; r++) {
        if (mode[r] != M_DONE && stat[r] == HRD_OK) {
            HRD_TRY(residual(r));
            stat[r] = HRD_ENOCONV;
        }
    }
    HRD_TRY(read_sc());
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int r = 0; r < total; r++) {
        if (stat[r] == HRD_ENOCONV) inf[r].true_rel_residual = std::sqrt(sc[(size_t)r * S_COUNT + S_RR]) / bnorm[r];
        inf[r].seconds = secs;
        if (infos) infos[r] = inf[r];
        if (stat[r] == HRD_EBREAKDOWN) result = HRD_EBREAKDOWN;
        else if (stat[r] == HRD_ENOCONV && result == HRD_OK) result = HRD_ENOCONV;
    }
    if (result == HRD_EBREAKDOWN) return fail(HRD_EBREAKDOWN, "breakdown in at least one right-hand side");
    if (result == HRD_ENOCONV) return fail(HRD_ENOCONV, "at least one right-hand side did not reach tol in %d iterations", maxiter);
    return HRD_OK;
#undef BT
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------

static std::string tune_key(const hrd_problem *probs, int nprob)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    std::string k = arch + "|batched_hop_f32";
    char buf[128];
    for (int i = 0; i < nprob; i++) {
        static const char *names[] = {"fund", "adj", "fund_su2", "adj_su2"};
        snprintf(buf, sizeof(buf), "|%dx%dx%dx%d/%s/%d", probs[i].lat.dims[0], probs[i].lat.dims[1], probs[i].lat.dims[2],
                 probs[i].lat.dims[3], names[probs[i].rep], probs[i].nrhs);
        k += buf;
    }
    return k;
}

static bool cache_lookup(const char *path, const std::string &key, hrd_tune *out)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    const std::string pat = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof(line), f)) {
        if (strstr(line, pat.c_str())) {
            hrd_tune t{};
            const char *p = strstr(line, "\"tune\": [");
            if (p && sscanf(p, "\"tune\": [%d, %d, %d, %d, %d]", &t.sites_per_tile, &t.rhs_per_tile,
                            &t.block_threads, &t.blocks_per_cu, &t.slab_width) == 5) {
                *out = t;
                found = true;
            }
        }
    }
    fclose(f);
    return found;
}

extern "C" hrd_status hrd_autotune_batched(const hrd_problem *probs, int nprob, void *work, size_t work_bytes,
                                const char *cache_path, hrd_tune *best, void *stream)
{
    HRD_TRY(check_problems(probs, nprob, false));
    if (!best) return fail(HRD_EINVAL, "NULL result");
    const std::string key = tune_key(probs, nprob);
    if (cache_path && cache_lookup(cache_path, key, best)) return HRD_OK;
    const hipStream_t st = (hipStream_t)stream;
    // the two timing events, destroyed on every return path
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    HRD_TRY(check_hip(hipEventCreate(&ev.e[0]), "hipEventCreate"));
    HRD_TRY(check_hip(hipEventCreate(&ev.e[1]), "hipEventCreate"));
    const int sites[] = {64, 128, 256};
    const int groups[] = {1, 2, 4, 6, 12};
    const int bpc[] = {2, 4, 8};
    const int slabs[] = {0, 1, 2, 4, 8, 1 << 20};  // 0: automatic; 1 << 20: whole L1 (lexicographic)
    float best_ms = 1e30f;
    hrd_tune bt{};
    for (int s : sites)
        for (int gsz : groups)
            for (int b : bpc)
                for (int sl : slabs) {
                    const hrd_tune cand{s, gsz, s, b, sl};
                    // one untimed launch, then the median of 5 timed ones; any
                    // failed launch or event call ends the search with its status
                    HRD_TRY(hrd_dirac_apply_batched(probs, nprob, HRD_EO, 0, &cand, work, work_bytes, stream));
                    float times[5];
                    for (int rep = 0; rep < 5; rep++) {
                        HRD_TRY(check_hip(hipEventRecord(ev.e[0], st), "hipEventRecord"));
                        HRD_TRY(hrd_dirac_apply_batched(probs, nprob, HRD_EO, 0, &cand, work, work_bytes, stream));
                        HRD_TRY(check_hip(hipEventRecord(ev.e[1], st), "hipEventRecord"));
                        HRD_TRY(check_hip(hipEventSynchronize(ev.e[1]), "hipEventSynchronize"));
                        HRD_TRY(check_hip(hipEventElapsedTime(&times[rep], ev.e[0], ev.e[1]), "hipEventElapsedTime"));
                    }
                    std::sort(times, times + 5);
                    const float med = times[2];
                    // ties (within 1%) go to the earlier, smaller candidate
                    if (med < best_ms * 0.99f) {
                        best_ms = med;
                        bt = cand;
                    }
                }
    *best = bt;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"tune\": [%d, %d, %d, %d, %d], \"median_ms\": %.6f}\n", key.c_str(),
                    bt.sites_per_tile, bt.rhs_per_tile, bt.block_threads, bt.blocks_per_cu, bt.slab_width, best_ms);
            fclose(f);
        }
    }
    return HRD_OK;
}
