// Clover (Sheikholeslami-Wohlert) site blocks: layout, loads/stores and the
// Hermitian block products used by the clover build kernel and the clover
// epilogues of the hopping kernel.
//
// In the chiral basis sigma_{mu nu} commutes with g5, so the site matrix
// M(x) = m + A(x) is block diagonal: an upper block acting on spins 0,1 and a
// lower block acting on spins 2,3, each a Hermitian 2N x 2N matrix (row index
// (spin - 2 b) N + colour).  A block is stored as its 2N real diagonal
// entries followed by the N(2N-1) complex entries below the diagonal in row
// order ((i, j) with i > j at position i(i-1)/2 + j): 4N^2 reals per block,
// 8N^2 per site.  A packed clover field is [parity][planes][Vh] with planes of
// 16-byte elements holding consecutive reals (two doubles or four floats).
#pragma once

#include "common.h"

namespace hrd {

__host__ __device__ constexpr int clover_site_reals(int n) { return 8 * n * n; }

template <int N, typename R>
struct CloverSite {
    R d[2][2 * N];
    Cx<R> l[2][N * (2 * N - 1)];
};

// One chirality block b of the site: its 4N^2 reals are F64 planes
// [2N^2 b, 2N^2 (b+1)) or F32 planes [N^2 b, N^2 (b+1)).
template <int N, typename R, bool NT = false>
__device__ __forceinline__ void clover_load_block(const void *C, int Vh, int p, int site, int b, R (&d)[2 * N],
                                                  Cx<R> (&l)[N * (2 * N - 1)])
{
    constexpr int K = clover_site_reals(N);
    constexpr int KB = K / 2;
    R e[KB];
    const char *base = reinterpret_cast<const char *>(C) + (size_t)p * Vh * K * sizeof(R);
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int q = 0; q < KB / 2; q++) {
            const vd2 v = ld16d<NT>(base + ((size_t)(b * KB / 2 + q) * Vh + site) * 16);
            e[2 * q] = v.x;
            e[2 * q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < KB / 4; q++) {
            const vf4 v = ld16f<NT>(base + ((size_t)(b * KB / 4 + q) * Vh + site) * 16);
            e[4 * q] = v.x;
            e[4 * q + 1] = v.y;
            e[4 * q + 2] = v.z;
            e[4 * q + 3] = v.w;
        }
    }
#pragma unroll
    for (int i = 0; i < 2 * N; i++) d[i] = e[i];
#pragma unroll
    for (int k = 0; k < N * (2 * N - 1); k++) l[k] = Cx<R>{e[2 * N + 2 * k], e[2 * N + 2 * k + 1]};
}

template <int N, typename R, bool NT = false>
__device__ __forceinline__ void clover_load(const void *C, int Vh, int p, int site, CloverSite<N, R> &c)
{
    clover_load_block<N, R, NT>(C, Vh, p, site, 0, c.d[0], c.l[0]);
    clover_load_block<N, R, NT>(C, Vh, p, site, 1, c.d[1], c.l[1]);
}

template <int N, typename R>
__device__ __forceinline__ void clover_store(void *C, int Vh, int p, int site, const CloverSite<N, R> &c)
{
    constexpr int K = clover_site_reals(N);
    R e[K];
#pragma unroll
    for (int b = 0; b < 2; b++) {
#pragma unroll
        for (int i = 0; i < 2 * N; i++) e[b * 4 * N * N + i] = c.d[b][i];
#pragma unroll
        for (int k = 0; k < N * (2 * N - 1); k++) {
            e[b * 4 * N * N + 2 * N + 2 * k] = c.l[b][k].re;
            e[b * 4 * N * N + 2 * N + 2 * k + 1] = c.l[b][k].im;
        }
    }
    char *base = reinterpret_cast<char *>(C) + (size_t)p * Vh * K * sizeof(R);
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int q = 0; q < K / 2; q++) st16d<false>(base + ((size_t)q * Vh + site) * 16, vd2{e[2 * q], e[2 * q + 1]});
    } else {
#pragma unroll
        for (int q = 0; q < K / 4; q++)
            st16f<false>(base + ((size_t)q * Vh + site) * 16, vf4{e[4 * q], e[4 * q + 1], e[4 * q + 2], e[4 * q + 3]});
    }
}

// y = M v for one Hermitian 2N x 2N block given as (diagonal, strict lower).
template <int N, typename R>
__device__ __forceinline__ void herm_block_mv(const R (&d)[2 * N], const Cx<R> (&l)[N * (2 * N - 1)],
                                              const Cx<R> *v, Cx<R> *y)
{
    constexpr int M = 2 * N;
#pragma unroll
    for (int i = 0; i < M; i++) {
        Cx<R> acc{d[i] * v[i].re, d[i] * v[i].im};
#pragma unroll
        for (int j = 0; j < M; j++) {
            if (j < i) acc = cfma(l[i * (i - 1) / 2 + j], v[j], acc);
            else if (j > i) acc = cfmac(l[j * (j - 1) / 2 + i], v[j], acc);
        }
        y[i] = acc;
    }
}

// out = M(x) v on a full spinor, reading the site's clover entries block by
// block from the packed field C (parity p, eo index site).
template <int N, typename R, bool NT = false>
__device__ __forceinline__ void clover_apply(const void *C, int Vh, int p, int site, const Cx<R> (&v)[4 * N],
                                             Cx<R> (&out)[4 * N])
{
#pragma unroll
    for (int b = 0; b < 2; b++) {
        R d[2 * N];
        Cx<R> l[N * (2 * N - 1)];
        clover_load_block<N, R, NT>(C, Vh, p, site, b, d, l);
        herm_block_mv<N, R>(d, l, v + 2 * N * b, out + 2 * N * b);
    }
}

}  // namespace hrd
