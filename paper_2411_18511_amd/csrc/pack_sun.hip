// Field preparation for SU(N > 2): natural <-> packed layouts of the dense
// link formats, precision conversion, and the fundamental, adjoint and
// two-index representations of fundamental SU(N) links (Sec. 1: SU(N) with
// fermions in higher representations; Sec. 2.2: derived fields computed once
// per gauge update).
//
// Bases (the operator's spectrum does not depend on them; these are fixed so
// results can be compared entry by entry):
//   adjoint   R_ab = 2 Re tr(T_a U T_b U^+), T_a the generalised Gell-Mann
//             matrices halved, ordered: for each pair j < k the symmetric
//             (E_jk + E_kj)/2 then the antisymmetric (-i E_jk + i E_kj)/2,
//             then the diagonal ones diag(1, .., 1, -l, 0, ..)/sqrt(2l(l+1)),
//             l = 1 .. N-1;
//   two-index the action M -> U M U^T on symmetric (antisymmetric) matrices in
//             the orthonormal basis E_(ij), i <= j (i < j), row-major:
//             e_i e_i^T and (e_i e_j^T +- e_j e_i^T)/sqrt(2);
//             R_kl = sum_xy (E_k)_xy (U E_l U^T)_xy.
#include "kernels.h"

namespace hrd {

namespace {

inline dim3 grid_for(long n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

template <int REP, typename S>
__global__ __launch_bounds__(kBlock) void pack_gauge_dense_kernel(Geom g, void *nat, void *packed, bool unpack)
{
    constexpr int N = ncolour(REP);
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long V = 2L * g.Vh;
    if (t >= 4 * V) return;
    const int mu = (int)(t / V);
    const long r = t - (long)mu * V;
    const int p = (int)(r / g.Vh);
    const int idx = (int)(r - (long)p * g.Vh);
    const Site s = eo_site(g, idx, p);
    using IO = LinkIO<REP, S>;
    if constexpr (is_real_dense(REP)) {
        double *e = reinterpret_cast<double *>(nat) + ((size_t)mu * V + s.lex) * N * N;
        if (!unpack) {
            RLink<N, double> l;
#pragma unroll
            for (int k = 0; k < N * N; k++) l.r[k / N][k % N] = e[k];
            IO::store(packed, g.Vh, p, mu, idx, l);
        } else {
            const auto l = IO::load(packed, g.Vh, p, mu, idx);
#pragma unroll
            for (int k = 0; k < N * N; k++) e[k] = (double)l.r[k / N][k % N];
        }
    } else {
        Cx<double> *e = reinterpret_cast<Cx<double> *>(nat) + ((size_t)mu * V + s.lex) * N * N;
        if (!unpack) {
            CLink<N, double> l;
#pragma unroll
            for (int k = 0; k < N * N; k++) l.u[k / N][k % N] = e[k];
            IO::store(packed, g.Vh, p, mu, idx, l);
        } else {
            const auto l = IO::load(packed, g.Vh, p, mu, idx);
#pragma unroll
            for (int k = 0; k < N * N; k++)
                e[k] = Cx<double>{(double)l.u[k / N][k % N].re, (double)l.u[k / N][k % N].im};
        }
    }
}

template <int REP, typename SO>
__global__ __launch_bounds__(kBlock) void convert_gauge_dense_kernel(Geom g, const void *U64, void *Uout)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    LinkIO<REP, SO>::store(Uout, g.Vh, p, mu, idx, LinkIO<REP, double>::load(U64, g.Vh, p, mu, idx));
}

// ---- representation maps -------------------------------------------------

template <int NC>
struct Mat {
    Cx<double> m[NC][NC];
};

template <int NC>
__device__ Mat<NC> matmul(const Mat<NC> &a, const Mat<NC> &b)
{
    Mat<NC> c;
    for (int i = 0; i < NC; i++)
        for (int j = 0; j < NC; j++) {
            Cx<double> z = cmul(a.m[i][0], b.m[0][j]);
            for (int k = 1; k < NC; k++) z = cfma(a.m[i][k], b.m[k][j], z);
            c.m[i][j] = z;
        }
    return c;
}

// Generator T_a of su(NC) in the order stated at the top of this file.
template <int NC>
__device__ Mat<NC> generator(int a)
{
    Mat<NC> t;
    for (int i = 0; i < NC; i++)
        for (int j = 0; j < NC; j++) t.m[i][j] = Cx<double>{0.0, 0.0};
    int c = 0;
    for (int j = 0; j < NC; j++)
        for (int k = j + 1; k < NC; k++) {
            if (c == a) {
                t.m[j][k] = t.m[k][j] = Cx<double>{0.5, 0.0};
                return t;
            }
            if (c + 1 == a) {
                t.m[j][k] = Cx<double>{0.0, -0.5};
                t.m[k][j] = Cx<double>{0.0, 0.5};
                return t;
            }
            c += 2;
        }
    const int l = a - c + 1;
    const double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
    for (int j = 0; j < l; j++) t.m[j][j] = Cx<double>{nrm, 0.0};
    t.m[l][l] = Cx<double>{-l * nrm, 0.0};
    return t;
}

// Two-index basis element k (SYM or not) as its index pair and sign.
template <int NC, bool SYM>
__device__ void basis_pair(int k, int &i, int &j)
{
    int c = 0;
    for (int a = 0; a < NC; a++)
        for (int b = SYM ? a : a + 1; b < NC; b++) {
            if (c == k) {
                i = a;
                j = b;
                return;
            }
            c++;
        }
    i = j = 0;
}

template <int NC, int KIND, int OUT>
__global__ __launch_bounds__(64) void represent_sun_kernel(Geom g, const void *Uf, void *Ur)
{
    constexpr int D = ncolour(OUT);
    const long t = (long)blockIdx.x * 64 + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    const auto f = CplxIO<NC, double>::load(Uf, g.Vh, p, mu, idx);
    Mat<NC> U, Ud;
    for (int i = 0; i < NC; i++)
        for (int j = 0; j < NC; j++) {
            U.m[i][j] = f.u[i][j];
            Ud.m[j][i] = Cx<double>{f.u[i][j].re, -f.u[i][j].im};
        }
    if constexpr (KIND == 0) {
        CLink<D, double> o;
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++) o.u[i][j] = U.m[i][j];
        LinkIO<OUT, double>::store(Ur, g.Vh, p, mu, idx, o);
    } else if constexpr (KIND == 1) {
        RLink<D, double> o;
        for (int b = 0; b < D; b++) {
            const Mat<NC> M = matmul(matmul(U, generator<NC>(b)), Ud);
            for (int a = 0; a < D; a++) {
                const Mat<NC> T = generator<NC>(a);
                double tr = 0.0;
                for (int x = 0; x < NC; x++)
                    for (int y = 0; y < NC; y++) tr += T.m[x][y].re * M.m[y][x].re - T.m[x][y].im * M.m[y][x].im;
                o.r[a][b] = 2.0 * tr;
            }
        }
        LinkIO<OUT, double>::store(Ur, g.Vh, p, mu, idx, o);
    } else {
        constexpr bool SYM = KIND == 2;
        const double r2 = 0.70710678118654752440;  // 1/sqrt(2)
        CLink<D, double> o;
        for (int l = 0; l < D; l++) {
            int a, b;
            basis_pair<NC, SYM>(l, a, b);
            // X = U E_l U^T: X_xy = w (U_xa U_yb +- U_xb U_ya) (w = 1/sqrt(2)), or U_xa U_ya for a = b
            for (int k = 0; k < D; k++) {
                int c, d;
                basis_pair<NC, SYM>(k, c, d);
                // R_kl = sum_xy (E_k)_xy X_xy: E_k has entries at (c, d) and (d, c)
                auto X = [&](int x, int y) {
                    if (a == b) return cmul(U.m[x][a], U.m[y][a]);
                    const Cx<double> s1 = cmul(U.m[x][a], U.m[y][b]), s2 = cmul(U.m[x][b], U.m[y][a]);
                    return SYM ? r2 * (s1 + s2) : r2 * (s1 - s2);
                };
                Cx<double> v;
                if (c == d) v = X(c, c);
                else v = SYM ? r2 * (X(c, d) + X(d, c)) : r2 * (X(c, d) - X(d, c));
                o.u[k][l] = v;
            }
        }
        LinkIO<OUT, double>::store(Ur, g.Vh, p, mu, idx, o);
    }
}

// Two-index basis element k as a dense matrix: e_c e_c^T, or
// (e_c e_d^T +- e_d e_c^T)/sqrt(2) for the pair (c, d) of basis_pair.
template <int NC, bool SYM>
__device__ Mat<NC> two_index_element(int k)
{
    Mat<NC> e;
    for (int i = 0; i < NC; i++)
        for (int j = 0; j < NC; j++) e.m[i][j] = Cx<double>{0.0, 0.0};
    int c, d;
    basis_pair<NC, SYM>(k, c, d);
    const double r2 = 0.70710678118654752440;  // 1/sqrt(2)
    if (c == d) {
        e.m[c][c] = Cx<double>{1.0, 0.0};
    } else {
        e.m[c][d] = Cx<double>{r2, 0.0};
        e.m[d][c] = Cx<double>{SYM ? r2 : -r2, 0.0};
    }
    return e;
}

// Chain rule of represent_sun_kernel: for L = Re sum conj(G) R(U) (real
// adjoint: L = sum G R(U)), Gf = dL/dRe U + i dL/dIm U:
//   fundamental: G;
//   adjoint:     R_ab = 2 tr(T_a U T_b U^+) gives 4 sum_ab G_ab T_a U T_b;
//   two-index:   R_kl = tr(E_k^T U E_l U^T) (E real, E^T = +-E) gives
//                dR_kl/dU = 2 E_k U E_l^T, so 2 sum_kl G_kl E_k conj(U) E_l^T.
template <int NC, int KIND, int RF>
__global__ __launch_bounds__(64) void represent_backward_sun_kernel(Geom g, const void *Uf, const void *Gr, void *Gf)
{
    constexpr int D = ncolour(RF);
    const long t = (long)blockIdx.x * 64 + threadIdx.x;
    if (t >= 8L * g.Vh) return;
    const int pm = (int)(t / g.Vh);
    const int idx = (int)(t - (long)pm * g.Vh);
    const int p = pm >> 2, mu = pm & 3;
    CLink<NC, double> out;
    if constexpr (KIND == 0) {
        out = CplxIO<NC, double>::load(Gr, g.Vh, p, mu, idx);
    } else {
        const auto f = CplxIO<NC, double>::load(Uf, g.Vh, p, mu, idx);
        Mat<NC> M, acc;  // M = U (adjoint) or conj(U) (two-index)
        for (int i = 0; i < NC; i++)
            for (int j = 0; j < NC; j++) {
                M.m[i][j] = KIND == 1 ? f.u[i][j] : Cx<double>{f.u[i][j].re, -f.u[i][j].im};
                acc.m[i][j] = Cx<double>{0.0, 0.0};
            }
        const auto G = LinkIO<RF, double>::load(Gr, g.Vh, p, mu, idx);
        for (int l = 0; l < D; l++) {
            // P = M B_l with B_l = T_l (adjoint) or E_l^T (two-index)
            Mat<NC> B;
            if constexpr (KIND == 1) {
                B = generator<NC>(l);
            } else {
                const Mat<NC> e = two_index_element<NC, KIND == 2>(l);
                for (int i = 0; i < NC; i++)
                    for (int j = 0; j < NC; j++) B.m[i][j] = e.m[j][i];
            }
            const Mat<NC> P = matmul(M, B);
            // A = sum_k c_kl A_k, A_k = T_k or E_k, c_kl = 4 G_kl or 2 G_kl
            Mat<NC> A;
            for (int i = 0; i < NC; i++)
                for (int j = 0; j < NC; j++) A.m[i][j] = Cx<double>{0.0, 0.0};
            for (int k = 0; k < D; k++) {
                const Mat<NC> Ak = KIND == 1 ? generator<NC>(k) : two_index_element<NC, KIND == 2>(k);
                Cx<double> c;
                if constexpr (KIND == 1) c = Cx<double>{4.0 * G.r[k][l], 0.0};
                else c = Cx<double>{2.0 * G.u[k][l].re, 2.0 * G.u[k][l].im};
                for (int i = 0; i < NC; i++)
                    for (int j = 0; j < NC; j++) A.m[i][j] = cfma(c, Ak.m[i][j], A.m[i][j]);
            }
            const Mat<NC> AP = matmul(A, P);
            for (int i = 0; i < NC; i++)
                for (int j = 0; j < NC; j++) acc.m[i][j] = acc.m[i][j] + AP.m[i][j];
        }
        for (int i = 0; i < NC; i++)
            for (int j = 0; j < NC; j++) out.u[i][j] = acc.m[i][j];
    }
    CplxIO<NC, double>::store(Gf, g.Vh, p, mu, idx, out);
}

template <typename S>
void pack_dense_for(int rep, const Geom &g, void *nat, void *packed, bool unpack, hipStream_t st)
{
    const dim3 grid = grid_for(8L * g.Vh);
    switch (rep) {
        case HRD_CPLX3: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_CPLX3, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        case HRD_CPLX4: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_CPLX4, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        case HRD_CPLX6: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_CPLX6, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        case HRD_CPLX10: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_CPLX10, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        case HRD_REAL15: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_REAL15, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        case HRD_SU3_ROW2: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_SU3_ROW2, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
        default: hipLaunchKernelGGL((pack_gauge_dense_kernel<HRD_REAL8, S>), grid, dim3(kBlock), 0, st, g, nat, packed, unpack); break;
    }
}

template <typename SO>
void convert_dense_for(int rep, const Geom &g, const void *U64, void *Uout, hipStream_t st)
{
    const dim3 grid = grid_for(8L * g.Vh);
    switch (rep) {
        case HRD_CPLX3: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_CPLX3, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        case HRD_CPLX4: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_CPLX4, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        case HRD_CPLX6: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_CPLX6, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        case HRD_CPLX10: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_CPLX10, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        case HRD_REAL15: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_REAL15, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        case HRD_SU3_ROW2: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_SU3_ROW2, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
        default: hipLaunchKernelGGL((convert_gauge_dense_kernel<HRD_REAL8, SO>), grid, dim3(kBlock), 0, st, g, U64, Uout); break;
    }
}

}  // namespace

hipError_t launch_pack_gauge_dense(int rep, int prec, const Geom &g, const void *nat, void *packed, bool unpack,
                                   hipStream_t st)
{
    void *n = const_cast<void *>(nat);
    switch (prec) {
        case HRD_F64: pack_dense_for<double>(rep, g, n, packed, unpack, st); break;
        case HRD_F32: pack_dense_for<float>(rep, g, n, packed, unpack, st); break;
        default: pack_dense_for<h16>(rep, g, n, packed, unpack, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_convert_gauge_dense(int rep, int prec_out, const Geom &g, const void *U64, void *Uout,
                                      hipStream_t st)
{
    if (prec_out == HRD_F32) convert_dense_for<float>(rep, g, U64, Uout, st);
    else convert_dense_for<h16>(rep, g, U64, Uout, st);
    return hipGetLastError();
}

hipError_t launch_represent_sun(int nc, int kind, const Geom &g, const void *Uf, void *Ur, hipStream_t st)
{
    const dim3 grid((unsigned)((8L * g.Vh + 63) / 64)), block(64);
    if (nc == 3) {
        switch (kind) {
            case 0: hipLaunchKernelGGL((represent_sun_kernel<3, 0, HRD_CPLX3>), grid, block, 0, st, g, Uf, Ur); break;
            case 1: hipLaunchKernelGGL((represent_sun_kernel<3, 1, HRD_REAL8>), grid, block, 0, st, g, Uf, Ur); break;
            case 2: hipLaunchKernelGGL((represent_sun_kernel<3, 2, HRD_CPLX6>), grid, block, 0, st, g, Uf, Ur); break;
            default: hipLaunchKernelGGL((represent_sun_kernel<3, 3, HRD_CPLX3>), grid, block, 0, st, g, Uf, Ur); break;
        }
    } else {
        switch (kind) {
            case 0: hipLaunchKernelGGL((represent_sun_kernel<4, 0, HRD_CPLX4>), grid, block, 0, st, g, Uf, Ur); break;
            case 1: hipLaunchKernelGGL((represent_sun_kernel<4, 1, HRD_REAL15>), grid, block, 0, st, g, Uf, Ur); break;
            case 2: hipLaunchKernelGGL((represent_sun_kernel<4, 2, HRD_CPLX10>), grid, block, 0, st, g, Uf, Ur); break;
            default: hipLaunchKernelGGL((represent_sun_kernel<4, 3, HRD_CPLX6>), grid, block, 0, st, g, Uf, Ur); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_represent_backward_sun(int nc, int kind, const Geom &g, const void *Uf, const void *Gr, void *Gf,
                                        hipStream_t st)
{
    const dim3 grid((unsigned)((8L * g.Vh + 63) / 64)), block(64);
    if (nc == 3) {
        switch (kind) {
            case 0: hipLaunchKernelGGL((represent_backward_sun_kernel<3, 0, HRD_CPLX3>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            case 1: hipLaunchKernelGGL((represent_backward_sun_kernel<3, 1, HRD_REAL8>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            case 2: hipLaunchKernelGGL((represent_backward_sun_kernel<3, 2, HRD_CPLX6>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            default: hipLaunchKernelGGL((represent_backward_sun_kernel<3, 3, HRD_CPLX3>), grid, block, 0, st, g, Uf, Gr, Gf); break;
        }
    } else {
        switch (kind) {
            case 0: hipLaunchKernelGGL((represent_backward_sun_kernel<4, 0, HRD_CPLX4>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            case 1: hipLaunchKernelGGL((represent_backward_sun_kernel<4, 1, HRD_REAL15>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            case 2: hipLaunchKernelGGL((represent_backward_sun_kernel<4, 2, HRD_CPLX10>), grid, block, 0, st, g, Uf, Gr, Gf); break;
            default: hipLaunchKernelGGL((represent_backward_sun_kernel<4, 3, HRD_CPLX6>), grid, block, 0, st, g, Uf, Gr, Gf); break;
        }
    }
    return hipGetLastError();
}

}  // namespace hrd
