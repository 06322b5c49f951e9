// Spin structure of the Wilson projectors (1 + SIG g_mu) in the chiral basis
// of hrd.h: the projector has rank 2, so (1 + SIG g_mu) psi is fixed by its
// upper two spin components h (a "half spinor"), and its lower two are
// SIG * g0-block h (mu = 0) or SIG i s_mu h (mu = 1..3).
#pragma once

#include "common.h"

namespace hrd {

// ca * x + cb * y with one fixed rounding sequence, fma(cb, y, ca * x), so
// every kernel that forms this combination produces identical bits.
template <typename R>
__device__ __forceinline__ Cx<R> axpby(R ca, Cx<R> x, R cb, Cx<R> y)
{
    return Cx<R>{fmadd(cb, y.re, ca * x.re), fmadd(cb, y.im, ca * x.im)};
}

template <int REP>
struct NCol {
    static constexpr int value = ncolour(REP);
};

// Upper half spinor of (1 + SIG g_mu) psi in the chiral basis.
// psi[k], k = spin * N + colour.
template <int MU, int SIG, int N, typename R>
__device__ __forceinline__ void project(const Cx<R> (&psi)[4 * N], Cx<R> (&h0)[N], Cx<R> (&h1)[N])
{
#pragma unroll
    for (int c = 0; c < N; c++) {
        const Cx<R> p0 = psi[c], p1 = psi[N + c], p2 = psi[2 * N + c], p3 = psi[3 * N + c];
        if constexpr (MU == 0) {  // h = psi_up + SIG psi_dn
            h0[c] = SIG > 0 ? p0 + p2 : p0 - p2;
            h1[c] = SIG > 0 ? p1 + p3 : p1 - p3;
        } else if constexpr (MU == 1) {  // h = psi_up - SIG i s1 psi_dn
            h0[c] = SIG > 0 ? p0 - mul_i(p3) : p0 + mul_i(p3);
            h1[c] = SIG > 0 ? p1 - mul_i(p2) : p1 + mul_i(p2);
        } else if constexpr (MU == 2) {  // h = psi_up - SIG i s2 psi_dn
            h0[c] = SIG > 0 ? p0 - p3 : p0 + p3;
            h1[c] = SIG > 0 ? p1 + p2 : p1 - p2;
        } else {  // h = psi_up - SIG i s3 psi_dn
            h0[c] = SIG > 0 ? p0 - mul_i(p2) : p0 + mul_i(p2);
            h1[c] = SIG > 0 ? p1 + mul_i(p3) : p1 - mul_i(p3);
        }
    }
}

// acc += (1 + SIG g_mu)-reconstruction of the colour-multiplied half spinor
// (u0, u1): upper = u, lower = SIG * g0-block (mu = 0) or SIG i s_mu u.
template <int MU, int SIG, int N, typename R>
__device__ __forceinline__ void reconstruct(Cx<R> (&acc)[4 * N], const Cx<R> (&u0)[N], const Cx<R> (&u1)[N])
{
#pragma unroll
    for (int c = 0; c < N; c++) {
        acc[c] = acc[c] + u0[c];
        acc[N + c] = acc[N + c] + u1[c];
        Cx<R> l2, l3;
        if constexpr (MU == 0) {
            l2 = u0[c];
            l3 = u1[c];
        } else if constexpr (MU == 1) {
            l2 = mul_i(u1[c]);
            l3 = mul_i(u0[c]);
        } else if constexpr (MU == 2) {
            l2 = u1[c];
            l3 = -u0[c];
        } else {
            l2 = mul_i(u0[c]);
            l3 = -mul_i(u1[c]);
        }
        if constexpr (SIG > 0) {
            acc[2 * N + c] = acc[2 * N + c] + l2;
            acc[3 * N + c] = acc[3 * N + c] + l3;
        } else {
            acc[2 * N + c] = acc[2 * N + c] - l2;
            acc[3 * N + c] = acc[3 * N + c] - l3;
        }
    }
}

}  // namespace hrd
