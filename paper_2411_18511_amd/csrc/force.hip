// Derivative of L = Re<X, D[U] Y> with respect to the links (the fermion
// force of the HMC that the paper's even/odd operator serves, Sec. 2.1):
//   G_mu(x) = -1/2 s_mu(x) sum_spin [ X(x) (x) ((1 - g_mu) Y(x+mu))^*
//                                   + ((1 + g_mu) Y(x)) (x) X(x+mu)^* ].
// Because (1 + SIG g_mu) is Hermitian, squares to twice itself and has the
// half-spinor structure of spin.h, each spin sum collapses to two spin
// components:  sum_s A_s (x) ((1+SIG g)B)_s^* = sum_{t=0,1} h(A)_t (x) h(B)_t^*
// with h the upper half of (1 + SIG g_mu) applied to the field.
// One thread per site computes the four links leaving it; every output link
// has exactly one writer (no atomics).  For the dense SU(N > 2) formats the
// derivative is written in the format itself (real part only for REAL8 and REAL15).
#include "kernels.h"
#include "spin.h"

namespace hrd {

namespace {

template <int MU, int REP>
__device__ __forceinline__ void force_dir(const Geom &g, const Site &s, int idx, int p, const char *Xb, const char *Yb,
                                          size_t half, const Cx<double> (&Xx)[4 * NCol<REP>::value],
                                          const Cx<double> (&Yx)[4 * NCol<REP>::value], void *F, double scale)
{
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    const int j = nbr_fwd(g, s, MU);
    const char *Xn = Xb + (size_t)(1 - p) * half;
    const char *Yn = Yb + (size_t)(1 - p) * half;
    Cx<double> Xf[NC], Yf[NC];
    SpinorIO<double>::template load<NC>(Xn, g.Vh, j, Xf);
    SpinorIO<double>::template load<NC>(Yn, g.Vh, j, Yf);
    // first term: (1 - g) projections of X(x) and Y(x+mu)
    Cx<double> a0[N], a1[N], b0[N], b1[N];
    project<MU, -1, N, double>(Xx, a0, a1);
    project<MU, -1, N, double>(Yf, b0, b1);
    // second term: (1 + g) projections of Y(x) and X(x+mu)
    Cx<double> c0[N], c1[N], d0[N], d1[N];
    project<MU, +1, N, double>(Yx, c0, c1);
    project<MU, +1, N, double>(Xf, d0, d1);
    const double sg = (MU == 0 && s.x[0] == g.L[0] - 1) ? -1.0 : 1.0;
    const double w = -0.5 * sg * scale;
    // G_ik = w (a_i conj(b_k) + a'_i conj(b'_k) + c_i conj(d_k) + c'_i conj(d'_k))
    auto entry = [&](int i, int k) {
        Cx<double> z = cmulc(b0[k], a0[i]);
        z = cfmac(b1[k], a1[i], z);
        z = cfmac(d0[k], c0[i], z);
        z = cfmac(d1[k], c1[i], z);
        return Cx<double>{w * z.re, w * z.im};
    };
    if constexpr (is_dense(REP)) {
        // dense formats, FP64 layout: entry e = N i + k in plane e (CPLXn:
        // one complex per plane) or in slot e % 2 of plane e / 2 (REALn: two
        // reals per plane; a row of odd length ends inside a plane and the
        // last plane of an odd entry count is padded with zero)
        char *blk = reinterpret_cast<char *>(F) +
                    (size_t)(4 * p + MU) * g.Vh * (size_t)link_bytes(REP, HRD_F64);
        if constexpr (is_real_dense(REP)) {
#pragma unroll
            for (int e = 0; e < N * N; e += 2) {
                const double v0 = entry(e / N, e % N).re;
                const double v1 = e + 1 < N * N ? entry((e + 1) / N, (e + 1) % N).re : 0.0;
                st16d<false>(blk + ((size_t)(e / 2) * g.Vh + idx) * 16, vd2{v0, v1});
            }
        } else {
#pragma unroll
            for (int i = 0; i < N; i++)
#pragma unroll
                for (int k = 0; k < N; k++) {
                    const Cx<double> z = entry(i, k);
                    st16d<false>(blk + ((size_t)(N * i + k) * g.Vh + idx) * 16, vd2{z.re, z.im});
                }
        }
    } else {
        Cx<double> G[N][N];
#pragma unroll
        for (int i = 0; i < N; i++)
#pragma unroll
            for (int k = 0; k < N; k++) G[i][k] = entry(i, k);
        if constexpr (base_rep(REP) == HRD_FUND) {
            FundLink<double> l;
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int k = 0; k < 2; k++) l.u[i][k] = G[i][k];
            LinkIO<HRD_FUND, double>::store(F, g.Vh, p, MU, idx, l);
        } else {
            AdjLink<double> l;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int k = 0; k < 3; k++) l.r[i][k] = G[i][k].re;
            LinkIO<HRD_ADJ, double>::store(F, g.Vh, p, MU, idx, l);
        }
    }
}

template <int REP>
__global__ __launch_bounds__(kBlock) void force_kernel(Geom g, const char *X, const char *Y, void *F, double scale)
{
    constexpr int N = NCol<REP>::value;
    constexpr int NC = 4 * N;
    int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int p = lb & 1;
    lb >>= 1;
    const int w = lb * kBlock + threadIdx.x;
    if (w >= g.Vh) return;
    const size_t half = (size_t)g.Vh * NC * sizeof(Cx<double>);
    int idx;
    const Site s = slab_site(g, w, p, &idx);
    Cx<double> Xx[NC], Yx[NC];
    SpinorIO<double>::template load<NC>(X + (size_t)p * half, g.Vh, idx, Xx);
    SpinorIO<double>::template load<NC>(Y + (size_t)p * half, g.Vh, idx, Yx);
    force_dir<0, REP>(g, s, idx, p, X, Y, half, Xx, Yx, F, scale);
    force_dir<1, REP>(g, s, idx, p, X, Y, half, Xx, Yx, F, scale);
    force_dir<2, REP>(g, s, idx, p, X, Y, half, Xx, Yx, F, scale);
    force_dir<3, REP>(g, s, idx, p, X, Y, half, Xx, Yx, F, scale);
}

}  // namespace

hipError_t launch_force(int rep, const Geom &g, const void *X, const void *Y, void *F, double scale, hipStream_t st)
{
    const dim3 grid(2 * ((g.Vh + kBlock - 1) / kBlock)), block(kBlock);
    const char *x = reinterpret_cast<const char *>(X);
    const char *y = reinterpret_cast<const char *>(Y);
    switch (base_rep(rep)) {
        case HRD_FUND: hipLaunchKernelGGL(force_kernel<HRD_FUND>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_ADJ: hipLaunchKernelGGL(force_kernel<HRD_ADJ>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_CPLX3: hipLaunchKernelGGL(force_kernel<HRD_CPLX3>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_CPLX4: hipLaunchKernelGGL(force_kernel<HRD_CPLX4>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_CPLX6: hipLaunchKernelGGL(force_kernel<HRD_CPLX6>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_CPLX10: hipLaunchKernelGGL(force_kernel<HRD_CPLX10>, grid, block, 0, st, g, x, y, F, scale); break;
        case HRD_REAL15: hipLaunchKernelGGL(force_kernel<HRD_REAL15>, grid, block, 0, st, g, x, y, F, scale); break;
        default: hipLaunchKernelGGL(force_kernel<HRD_REAL8>, grid, block, 0, st, g, x, y, F, scale); break;
    }
    return hipGetLastError();
}

}  // namespace hrd
