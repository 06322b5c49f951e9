// Clover term of the improved Wilson operator (the paper's Sec. 2.2: an
// extra site-diagonal term, for the SU(2) formats and SU(3) fundamental links
// (CPLX3, SU3_ROW2), whose derived fields are precomputed once per
// gauge field).  One thread per site builds
//   M(x) = m + A(x),  A(x) = c_sw (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu}(x),
// with F the four-leaf field strength (Q - Q^+)/8, and its inverse, which the
// hopping kernel then applies in its epilogues (M on even sites and M^{-1} on
// odd sites of the even/odd operator).  In the chiral basis
//   sigma_{0k} = diag(-s_k, +s_k),   sigma_{jk} = -eps_{jkl} diag(s_l, s_l),
// so with B_l = F_{0l} and E = (F_23, -F_13, F_12):
//   A_up = -sum_l s_l (x) X_l,  X_l = c_sw (i/2)(B_l + E_l),
//   A_dn = +sum_l s_l (x) Y_l,  Y_l = c_sw (i/2)(B_l - E_l).
// The paper stores an LDL factorisation; here the inverse blocks themselves
// are stored, so applying M^{-1} costs the same as applying M.
//
// The exponentiated variant (also named in Sec. 2.2) replaces m + A by
// M = m exp(A/m), whose inverse (1/m) exp(-A/m) is again an exponential; each
// Hermitian block is exponentiated by scaling and squaring around a Taylor
// polynomial (X / 2^s with ||X / 2^s||_1 <= 1/4, degree 16: truncation below
// 1e-24 relative before squaring).
#include "clover.h"
#include "kernels.h"

namespace hrd {

namespace {

template <int N>
struct CMat {
    Cx<double> m[N][N];
};

template <int N>
__device__ __forceinline__ CMat<N> mm(const CMat<N> &a, const CMat<N> &b)
{
    CMat<N> c;
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            Cx<double> z = cmul(a.m[i][0], b.m[0][j]);
#pragma unroll
            for (int k = 1; k < N; k++) z = cfma(a.m[i][k], b.m[k][j], z);
            c.m[i][j] = z;
        }
    return c;
}

template <int N>
__device__ __forceinline__ CMat<N> dag(const CMat<N> &a)
{
    CMat<N> c;
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) c.m[i][j] = Cx<double>{a.m[j][i].re, -a.m[j][i].im};
    return c;
}

__device__ __forceinline__ CMat<2> as_mat(const FundLink<double> &l)
{
    CMat<2> c;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) c.m[i][j] = l.u[i][j];
    return c;
}

template <int N>
__device__ __forceinline__ CMat<N> as_mat(const CLink<N, double> &l)
{
    CMat<N> c;
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) c.m[i][j] = l.u[i][j];
    return c;
}

__device__ __forceinline__ CMat<3> as_mat(const AdjLink<double> &l)
{
    CMat<3> c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.m[i][j] = Cx<double>{l.r[i][j], 0.0};
    return c;
}

// Link U_mu at the site with coordinates x (periodic wrap applied by the caller).
template <int REP>
__device__ __forceinline__ CMat<ncolour(REP)> link_at(const void *U, const Geom &g, const int (&x)[4], int mu)
{
    const int lex = ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    return as_mat(LinkIO<REP, double>::load(U, g.Vh, p, mu, lex >> 1));
}

__device__ __forceinline__ void shift2(const Geom &g, const int (&x)[4], int mu, int dm, int nu, int dn, int (&y)[4])
{
#pragma unroll
    for (int k = 0; k < 4; k++) y[k] = x[k];
    y[mu] = (y[mu] + dm + g.L[mu]) % g.L[mu];
    y[nu] = (y[nu] + dn + g.L[nu]) % g.L[nu];
}

// F_{mu nu}(x) = (Q - Q^+) / 8, Q the four same-oriented leaves at x.
template <int REP>
__device__ CMat<ncolour(REP)> field_strength(const void *U, const Geom &g, const int (&x)[4], int mu, int nu)
{
    constexpr int N = ncolour(REP);
    int a[4], b[4], c[4];
    // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    shift2(g, x, mu, 1, nu, 0, a);
    shift2(g, x, mu, 0, nu, 1, b);
    CMat<N> Q = mm(mm(mm(link_at<REP>(U, g, x, mu), link_at<REP>(U, g, a, nu)), dag(link_at<REP>(U, g, b, mu))),
                   dag(link_at<REP>(U, g, x, nu)));
    // U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    shift2(g, x, mu, -1, nu, 1, a);
    shift2(g, x, mu, -1, nu, 0, b);
    CMat<N> L = mm(mm(mm(link_at<REP>(U, g, x, nu), dag(link_at<REP>(U, g, a, mu))), dag(link_at<REP>(U, g, b, nu))),
                   link_at<REP>(U, g, b, mu));
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) Q.m[i][j] = Q.m[i][j] + L.m[i][j];
    // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    shift2(g, x, mu, -1, nu, 0, a);
    shift2(g, x, mu, -1, nu, -1, b);
    shift2(g, x, mu, 0, nu, -1, c);
    L = mm(mm(mm(dag(link_at<REP>(U, g, a, mu)), dag(link_at<REP>(U, g, b, nu))), link_at<REP>(U, g, b, mu)),
           link_at<REP>(U, g, c, nu));
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) Q.m[i][j] = Q.m[i][j] + L.m[i][j];
    // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    shift2(g, x, mu, 0, nu, -1, a);
    shift2(g, x, mu, 1, nu, -1, b);
    L = mm(mm(mm(dag(link_at<REP>(U, g, a, nu)), link_at<REP>(U, g, a, mu)), link_at<REP>(U, g, b, nu)),
           dag(link_at<REP>(U, g, x, mu)));
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) Q.m[i][j] = Q.m[i][j] + L.m[i][j];
    CMat<N> F;
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++)
            F.m[i][j] = Cx<double>{0.125 * (Q.m[i][j].re - Q.m[j][i].re), 0.125 * (Q.m[i][j].im + Q.m[j][i].im)};
    return F;
}

// c (i/2) z
__device__ __forceinline__ Cx<double> ihalf(double c, Cx<double> z) { return Cx<double>{-0.5 * c * z.im, 0.5 * c * z.re}; }

// In-place inverse of a complex M x M matrix, Gauss-Jordan with partial pivoting.
template <int M>
__device__ void invert(Cx<double> (&a)[M][M])
{
    Cx<double> inv[M][M];
#pragma unroll
    for (int i = 0; i < M; i++)
#pragma unroll
        for (int j = 0; j < M; j++) inv[i][j] = Cx<double>{i == j ? 1.0 : 0.0, 0.0};
    for (int k = 0; k < M; k++) {
        int piv = k;
        double best = a[k][k].re * a[k][k].re + a[k][k].im * a[k][k].im;
        for (int i = k + 1; i < M; i++) {
            const double v = a[i][k].re * a[i][k].re + a[i][k].im * a[i][k].im;
            if (v > best) {
                best = v;
                piv = i;
            }
        }
        if (piv != k)
            for (int j = 0; j < M; j++) {
                const Cx<double> t = a[k][j];
                a[k][j] = a[piv][j];
                a[piv][j] = t;
                const Cx<double> u = inv[k][j];
                inv[k][j] = inv[piv][j];
                inv[piv][j] = u;
            }
        const Cx<double> pk = a[k][k];
        const double n2 = pk.re * pk.re + pk.im * pk.im;
        const Cx<double> r{pk.re / n2, -pk.im / n2};
        for (int j = 0; j < M; j++) {
            a[k][j] = cmul(r, a[k][j]);
            inv[k][j] = cmul(r, inv[k][j]);
        }
        for (int i = 0; i < M; i++) {
            if (i == k) continue;
            const Cx<double> f = a[i][k];
            for (int j = 0; j < M; j++) {
                a[i][j] = a[i][j] - cmul(f, a[k][j]);
                inv[i][j] = inv[i][j] - cmul(f, inv[k][j]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < M; i++)
#pragma unroll
        for (int j = 0; j < M; j++) a[i][j] = inv[i][j];
}

// E = exp(c X) for a 2N x 2N block X (c = +-1/m), scaling and squaring.
template <int M>
__device__ void expm_block(const Cx<double> (&X)[M][M], double c, Cx<double> (&E)[M][M])
{
    double nrm = 0.0;
    for (int j = 0; j < M; j++) {
        double col = 0.0;
        for (int i = 0; i < M; i++) col += fabs(X[i][j].re) + fabs(X[i][j].im);
        nrm = fmax(nrm, col);
    }
    nrm *= fabs(c);
    int sq = 0;
    while (nrm > 0.25 && sq < 64) {
        nrm *= 0.5;
        sq++;
    }
    const double scale = ldexp(c, -sq);
    Cx<double> Y[M][M], T[M][M];
    for (int i = 0; i < M; i++)
        for (int j = 0; j < M; j++) {
            Y[i][j] = scale * X[i][j];
            E[i][j] = Cx<double>{i == j ? 1.0 : 0.0, 0.0};
        }
    // Horner: E = I + Y/1 (I + Y/2 (... (I + Y/16)))
    constexpr int kDegree = 16;
    for (int k = kDegree; k >= 1; k--) {
        const double rk = 1.0 / k;
        for (int i = 0; i < M; i++)
            for (int j = 0; j < M; j++) {
                Cx<double> z = cmul(Y[i][0], E[0][j]);
                for (int l = 1; l < M; l++) z = cfma(Y[i][l], E[l][j], z);
                T[i][j] = rk * z;
            }
        for (int i = 0; i < M; i++)
            for (int j = 0; j < M; j++) E[i][j] = Cx<double>{(i == j ? 1.0 : 0.0) + T[i][j].re, T[i][j].im};
    }
    for (int q = 0; q < sq; q++) {
        for (int i = 0; i < M; i++)
            for (int j = 0; j < M; j++) {
                Cx<double> z = cmul(E[i][0], E[0][j]);
                for (int l = 1; l < M; l++) z = cfma(E[i][l], E[l][j], z);
                T[i][j] = z;
            }
        for (int i = 0; i < M; i++)
            for (int j = 0; j < M; j++) E[i][j] = T[i][j];
    }
}

template <int N>
__device__ __forceinline__ void pack_block(const Cx<double> (&a)[2 * N][2 * N], double (&d)[2 * N],
                                           Cx<double> (&l)[N * (2 * N - 1)])
{
#pragma unroll
    for (int i = 0; i < 2 * N; i++) {
        d[i] = a[i][i].re;
#pragma unroll
        for (int j = 0; j < i; j++) l[i * (i - 1) / 2 + j] = a[i][j];
    }
}

template <int REP, bool EXP>
__global__ __launch_bounds__(64) void clover_build_kernel(Geom g, const void *U, double csw, double m, void *Mf,
                                                          void *Mi)
{
    constexpr int N = ncolour(REP);
    constexpr int B2 = 2 * N;
    const long t = (long)blockIdx.x * 64 + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    const int p = (int)(t / g.Vh);
    const int idx = (int)(t - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    int x[4] = {s.x[0], s.x[1], s.x[2], s.x[3]};
    CMat<N> Bf[3], E[3];
    for (int l = 0; l < 3; l++) Bf[l] = field_strength<REP>(U, g, x, 0, l + 1);
    E[0] = field_strength<REP>(U, g, x, 2, 3);
    E[1] = field_strength<REP>(U, g, x, 1, 3);
    E[2] = field_strength<REP>(U, g, x, 1, 2);
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) E[1].m[i][j] = -E[1].m[i][j];
    Cx<double> up[B2][B2], dn[B2][B2];
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int j = 0; j < N; j++) {
            Cx<double> X[3], Y[3];
#pragma unroll
            for (int l = 0; l < 3; l++) {
                X[l] = ihalf(csw, Bf[l].m[i][j] + E[l].m[i][j]);
                Y[l] = ihalf(csw, Bf[l].m[i][j] - E[l].m[i][j]);
            }
            // s1 (x) X1 + s2 (x) X2 + s3 (x) X3 = [[X3, X1 - i X2], [X1 + i X2, -X3]]
            const Cx<double> iX2 = mul_i(X[1]), iY2 = mul_i(Y[1]);
            up[i][j] = -X[2];
            up[i][N + j] = -(X[0] - iX2);
            up[N + i][j] = -(X[0] + iX2);
            up[N + i][N + j] = X[2];
            dn[i][j] = Y[2];
            dn[i][N + j] = Y[0] - iY2;
            dn[N + i][j] = Y[0] + iY2;
            dn[N + i][N + j] = -Y[2];
        }
    CloverSite<N, double> c;
    if constexpr (EXP) {
        Cx<double> E[B2][B2];
        expm_block<B2>(up, 1.0 / m, E);
        for (int i = 0; i < B2; i++)
            for (int j = 0; j < B2; j++) E[i][j] = m * E[i][j];
        pack_block<N>(E, c.d[0], c.l[0]);
        expm_block<B2>(dn, 1.0 / m, E);
        for (int i = 0; i < B2; i++)
            for (int j = 0; j < B2; j++) E[i][j] = m * E[i][j];
        pack_block<N>(E, c.d[1], c.l[1]);
        clover_store<N, double>(Mf, g.Vh, p, idx, c);
        const double rm = 1.0 / m;
        expm_block<B2>(up, -rm, E);
        for (int i = 0; i < B2; i++)
            for (int j = 0; j < B2; j++) E[i][j] = rm * E[i][j];
        pack_block<N>(E, c.d[0], c.l[0]);
        expm_block<B2>(dn, -rm, E);
        for (int i = 0; i < B2; i++)
            for (int j = 0; j < B2; j++) E[i][j] = rm * E[i][j];
        pack_block<N>(E, c.d[1], c.l[1]);
        clover_store<N, double>(Mi, g.Vh, p, idx, c);
    } else {
#pragma unroll
        for (int i = 0; i < B2; i++) {
            up[i][i].re += m;
            dn[i][i].re += m;
        }
        pack_block<N>(up, c.d[0], c.l[0]);
        pack_block<N>(dn, c.d[1], c.l[1]);
        clover_store<N, double>(Mf, g.Vh, p, idx, c);
        invert<B2>(up);
        invert<B2>(dn);
        pack_block<N>(up, c.d[0], c.l[0]);
        pack_block<N>(dn, c.d[1], c.l[1]);
        clover_store<N, double>(Mi, g.Vh, p, idx, c);
    }
}

// F64 -> F32 packed clover field: real r of a site lives in F64 plane r/2 and
// F32 plane r/4; one thread per (parity, F32 plane, site).
__global__ __launch_bounds__(kBlock) void convert_clover_kernel(int Vh, int K, const double *c64, float *c32)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const int np32 = K / 4;
    if (t >= 2L * np32 * Vh) return;
    const int p = (int)(t / ((long)np32 * Vh));
    const long r = t - (long)p * np32 * Vh;
    const int q = (int)(r / Vh);
    const int site = (int)(r - (long)q * Vh);
    const double *b64 = c64 + (size_t)p * Vh * K;
    float *b32 = c32 + (size_t)p * Vh * K;
    const double2 a = reinterpret_cast<const double2 *>(b64)[(size_t)(2 * q) * Vh + site];
    const double2 b = reinterpret_cast<const double2 *>(b64)[(size_t)(2 * q + 1) * Vh + site];
    reinterpret_cast<float4 *>(b32)[(size_t)q * Vh + site] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

// Packed F64 clover field -> natural complex128 [V][4N][4N] (full Hermitian blocks).
template <int N>
__global__ __launch_bounds__(kBlock) void unpack_clover_kernel(Geom g, const void *C, Cx<double> *nat)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 2L * g.Vh) return;
    const int p = (int)(t / g.Vh);
    const int idx = (int)(t - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    CloverSite<N, double> c;
    clover_load<N, double>(C, g.Vh, p, idx, c);
    constexpr int D = 4 * N;
    Cx<double> *o = nat + (size_t)s.lex * D * D;
    for (int k = 0; k < D * D; k++) o[k] = Cx<double>{0.0, 0.0};
    for (int b = 0; b < 2; b++)
        for (int i = 0; i < 2 * N; i++)
            for (int j = 0; j < 2 * N; j++) {
                Cx<double> v;
                if (i == j) v = Cx<double>{c.d[b][i], 0.0};
                else if (i > j) v = c.l[b][i * (i - 1) / 2 + j];
                else v = Cx<double>{c.l[b][j * (j - 1) / 2 + i].re, -c.l[b][j * (j - 1) / 2 + i].im};
                o[(2 * N * b + i) * D + 2 * N * b + j] = v;
            }
}

}  // namespace

template <bool EXP>
hipError_t launch_build(int rep, const Geom &g, const void *U, double csw, double m, void *Mf, void *Mi,
                        hipStream_t st)
{
    const dim3 grid((unsigned)((2L * g.Vh + 63) / 64)), block(64);
    switch (rep) {
        case HRD_FUND:
            hipLaunchKernelGGL((clover_build_kernel<HRD_FUND, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
        case HRD_ADJ:
            hipLaunchKernelGGL((clover_build_kernel<HRD_ADJ, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
        case HRD_FUND_SU2:
            hipLaunchKernelGGL((clover_build_kernel<HRD_FUND_SU2, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
        case HRD_CPLX3:
            hipLaunchKernelGGL((clover_build_kernel<HRD_CPLX3, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
        case HRD_SU3_ROW2:
            hipLaunchKernelGGL((clover_build_kernel<HRD_SU3_ROW2, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
        default:
            hipLaunchKernelGGL((clover_build_kernel<HRD_ADJ_SU2, EXP>), grid, block, 0, st, g, U, csw, m, Mf, Mi);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_clover_build(int rep, bool exponential, const Geom &g, const void *U, double csw, double m, void *Mf,
                               void *Mi, hipStream_t st)
{
    return exponential ? launch_build<true>(rep, g, U, csw, m, Mf, Mi, st)
                       : launch_build<false>(rep, g, U, csw, m, Mf, Mi, st);
}

hipError_t launch_convert_clover(int rep, const Geom &g, const void *C64, void *C32, hipStream_t st)
{
    const int K = clover_site_reals(ncolour(rep));
    const long n = 2L * (K / 4) * g.Vh;
    hipLaunchKernelGGL(convert_clover_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, g.Vh, K,
                       (const double *)C64, (float *)C32);
    return hipGetLastError();
}

hipError_t launch_unpack_clover(int rep, const Geom &g, const void *C, void *nat, hipStream_t st)
{
    const dim3 grid((unsigned)((2L * g.Vh + kBlock - 1) / kBlock)), block(kBlock);
    if (ncolour(rep) == 2) hipLaunchKernelGGL(unpack_clover_kernel<2>, grid, block, 0, st, g, C, (Cx<double> *)nat);
    else hipLaunchKernelGGL(unpack_clover_kernel<3>, grid, block, 0, st, g, C, (Cx<double> *)nat);
    return hipGetLastError();
}

}  // namespace hrd
