/*
 * Oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU evaluation of the Wilson-Dirac
 * hopping term, the adjoint-representation map, the derivative of
 * Re<X, D[U] Y> with respect to the links, and the plaquette, for SU(2)
 * gauge fields.  It exists to check the GPU library; only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code with the GPU library.
 *
 * The paper (arXiv:2411.18511, "Scaling SU(2) to 1000 GPUs using HiRep",
 * Sec. 2.1 and Table 1) names the unimproved Wilson-Dirac operator with
 * SU(2) links in the fundamental and in higher representations, but never
 * writes it down.  The definitions used here are the textbook ones, fixed as
 * follows (every choice is a reading of a silent paper):
 *
 *   Lattice  x = (t, x1, x2, x3), extents (T, L1, L2, L3); mu = 0 is time.
 *            lex(x) = ((t*L1 + x1)*L2 + x2)*L3 + x3.
 *   Fields   U[mu][lex][i][j]  (N x N complex, N = 2 fund, 3 adjoint with
 *            zero imaginary part), psi[lex][spin][colour] (4 x N complex).
 *   Gammas   chiral basis, 2x2 blocks: g0 = [[0,1],[1,0]],
 *            gk = [[0,-i s_k],[i s_k,0]] with Pauli matrices s_k.
 *   Boundary periodic in space, antiperiodic in time, carried by the hop
 *            sign s_mu(x) = -1 iff mu = 0 and t(x) = T-1 (links stay periodic).
 *   Hopping  (H psi)(x) = sum_mu [ s_mu(x) (1 - g_mu) U_mu(x) psi(x+mu)
 *                               + s_mu(x-mu) (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   Operator D = (4 + m0) - H/2.
 *
 * Every function below evaluates those sums literally, with full 4x4 gamma
 * matrices and no spin-projection shortcut.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define MAXN 16

/* Coordinates of lexicographic site index s. */
static void coords(const int *d, long s, int x[4])
{
    x[3] = (int)(s % d[3]); s /= d[3];
    x[2] = (int)(s % d[2]); s /= d[2];
    x[1] = (int)(s % d[1]); s /= d[1];
    x[0] = (int)s;
}

static long lexidx(const int *d, const int x[4])
{
    return (((long)x[0] * d[1] + x[1]) * d[2] + x[2]) * d[3] + x[3];
}

static long volume(const int *d) { return (long)d[0] * d[1] * d[2] * d[3]; }

/* The four Euclidean gamma matrices of the chiral basis (see header). */
static void gamma_matrix(int mu, cplx g[4][4])
{
    /* Pauli matrices s1, s2, s3 */
    const cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(g, 0, sizeof(cplx) * 16);
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            if (mu == 0) {
                g[a][2 + b] = (a == b) ? 1 : 0;
                g[2 + a][b] = (a == b) ? 1 : 0;
            } else {
                g[a][2 + b] = -I * pauli[mu - 1][a][b];
                g[2 + a][b] = I * pauli[mu - 1][a][b];
            }
        }
}

/* Exported so the tests can check the Clifford algebra of the basis used. */
void oracle_gamma(int mu, cplx *out)
{
    cplx g[4][4];
    gamma_matrix(mu, g);
    memcpy(out, g, sizeof(g));
}

/* Hop sign s_mu(x) for the time-antiperiodic boundary. */
static double hop_sign(const int *d, int mu, const int x[4])
{
    return (mu == 0 && x[0] == d[0] - 1) ? -1.0 : 1.0;
}

/*
 * out(x) = (H psi)(x) on the sites whose parity bit is set in `mask`
 * (bit 0: even sites, bit 1: odd sites); every other site of `out` is set
 * to zero.  Parity of x is (t + x1 + x2 + x3) mod 2.
 */
void oracle_hopping(const int *d, int n, const cplx *U, const cplx *psi,
                    cplx *out, int mask)
{
    const long V = volume(d);
    cplx G[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
        cplx acc[4][MAXN];
        memset(acc, 0, sizeof(acc));
        if (mask & (1 << par)) {
            for (int mu = 0; mu < 4; mu++) {
                int y[4];
                cplx v[4][MAXN];

                /* forward term: s_mu(x) (1 - g_mu) U_mu(x) psi(x + mu) */
                memcpy(y, x, sizeof(y));
                y[mu] = (x[mu] + 1) % d[mu];
                const long sf = lexidx(d, y);
                const double sgf = hop_sign(d, mu, x);
                const cplx *Uf = U + ((long)mu * V + s) * n * n;
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < n; i++) {
                        cplx z = 0;
                        for (int j = 0; j < n; j++)
                            z += Uf[i * n + j] * psi[(sf * 4 + a) * n + j];
                        v[a][i] = z;
                    }
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < n; i++) {
                        cplx z = v[a][i];
                        for (int b = 0; b < 4; b++) z -= G[mu][a][b] * v[b][i];
                        acc[a][i] += sgf * z;
                    }

                /* backward term: s_mu(x-mu) (1 + g_mu) U_mu(x-mu)^+ psi(x - mu) */
                memcpy(y, x, sizeof(y));
                y[mu] = (x[mu] - 1 + d[mu]) % d[mu];
                const long sb = lexidx(d, y);
                const double sgb = hop_sign(d, mu, y);
                const cplx *Ub = U + ((long)mu * V + sb) * n * n;
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < n; i++) {
                        cplx z = 0;
                        for (int j = 0; j < n; j++)
                            z += conj(Ub[j * n + i]) * psi[(sb * 4 + a) * n + j];
                        v[a][i] = z;
                    }
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < n; i++) {
                        cplx z = v[a][i];
                        for (int b = 0; b < 4; b++) z += G[mu][a][b] * v[b][i];
                        acc[a][i] += sgb * z;
                    }
            }
        }
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < n; i++) out[(s * 4 + a) * n + i] = acc[a][i];
    }
}

/* out = (4 + m0) psi - H psi / 2 on all sites. */
void oracle_dirac(const int *d, int n, const cplx *U, const cplx *psi,
                  cplx *out, double m0)
{
    const long V = volume(d);
    oracle_hopping(d, n, U, psi, out, 3);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V * 4 * n; k++)
        out[k] = (4.0 + m0) * psi[k] - 0.5 * out[k];
}

/*
 * Adjoint representation of SU(2): R_ab(U) = (1/2) tr(s_a U s_b U^+),
 * a, b = 1..3, a real 3x3 matrix.  Uf is [nlinks][2][2], R is [nlinks][3][3].
 */
void oracle_represent_adjoint(long nlinks, const cplx *Uf, double *R)
{
    const cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nlinks; l++) {
        const cplx *u = Uf + l * 4;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                /* tr(s_a U s_b U^+) = sum_{ijkm} s_a[i][j] U[j][k] s_b[k][m] conj(U[i][m]) */
                cplx tr = 0;
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 2; j++)
                        for (int k = 0; k < 2; k++)
                            for (int m = 0; m < 2; m++)
                                tr += pauli[a][i][j] * u[j * 2 + k] * pauli[b][k][m] *
                                      conj(u[i * 2 + m]);
                R[l * 9 + a * 3 + b] = 0.5 * creal(tr);
            }
    }
}

/*
 * Derivative of L = Re<X, D[U] Y> with respect to the links, in the
 * convention G = dL/dRe(U) + i dL/dIm(U) for each entry of U_mu(x).
 * D depends on U only through the hopping term, linearly, so G depends on
 * X and Y alone:
 *   G_mu(x)_ij = -1/2 s_mu(x) sum_spin [ X(x)_{s,i} conj(((1 - g_mu) Y(x+mu))_{s,j})
 *                                      + ((1 + g_mu) Y(x))_{s,i} conj(X(x+mu)_{s,j}) ]
 * (the first sum comes from the forward term at x, the second from the
 * backward term at x + mu, which also uses U_mu(x)).  G is [mu][lex][i][j].
 */
void oracle_force(const int *d, int n, const cplx *X, const cplx *Y, cplx *Gout)
{
    const long V = volume(d);
    cplx G[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        for (int mu = 0; mu < 4; mu++) {
            int y[4];
            memcpy(y, x, sizeof(y));
            y[mu] = (x[mu] + 1) % d[mu];
            const long sf = lexidx(d, y);
            const double sg = hop_sign(d, mu, x);
            cplx pm[4][MAXN], pp[4][MAXN];
            /* pm = (1 - g_mu) Y(x+mu),  pp = (1 + g_mu) Y(x) */
            for (int a = 0; a < 4; a++)
                for (int i = 0; i < n; i++) {
                    cplx zm = Y[(sf * 4 + a) * n + i];
                    cplx zp = Y[(s * 4 + a) * n + i];
                    for (int b = 0; b < 4; b++) {
                        zm -= G[mu][a][b] * Y[(sf * 4 + b) * n + i];
                        zp += G[mu][a][b] * Y[(s * 4 + b) * n + i];
                    }
                    pm[a][i] = zm;
                    pp[a][i] = zp;
                }
            cplx *g = Gout + ((long)mu * V + s) * n * n;
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++) {
                    cplx z = 0;
                    for (int a = 0; a < 4; a++)
                        z += X[(s * 4 + a) * n + i] * conj(pm[a][j]) +
                             pp[a][i] * conj(X[(sf * 4 + a) * n + j]);
                    g[i * n + j] = -0.5 * sg * z;
                }
        }
    }
}

/*
 * Average plaquette (1/N) Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
 * over all sites and the six planes mu < nu.
 */
double oracle_plaquette(const int *d, int n, const cplx *U)
{
    const long V = volume(d);
    double total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                int y[4];
                memcpy(y, x, sizeof(y));
                y[mu] = (x[mu] + 1) % d[mu];
                const long sxm = lexidx(d, y);
                memcpy(y, x, sizeof(y));
                y[nu] = (x[nu] + 1) % d[nu];
                const long sxn = lexidx(d, y);
                const cplx *A = U + ((long)mu * V + s) * n * n;
                const cplx *B = U + ((long)nu * V + sxm) * n * n;
                const cplx *C = U + ((long)mu * V + sxn) * n * n;
                const cplx *E = U + ((long)nu * V + s) * n * n;
                cplx tr = 0;
                for (int i = 0; i < n; i++)
                    for (int j = 0; j < n; j++)
                        for (int k = 0; k < n; k++)
                            for (int l = 0; l < n; l++)
                                tr += A[i * n + j] * B[j * n + k] * conj(C[l * n + k]) *
                                      conj(E[i * n + l]);
                total += creal(tr) / n;
            }
    }
    return total / (6.0 * V);
}

/*
 * Clover (Sheikholeslami-Wohlert) term, Sec. 2.2 of the paper ("another
 * diagonal term" of the improved operator; the paper gives no formula).
 * Reading: the standard one,
 *   A(x) = c_sw (i/4) sum_{mu,nu} sigma_{mu nu} (x) F_{mu nu}(x),
 *   sigma_{mu nu} = (i/2) [g_mu, g_nu],
 *   F_{mu nu}(x) = (1/8) [Q_{mu nu}(x) - Q_{mu nu}(x)^+],
 * with Q_{mu nu}(x) the sum of the four plaquettes of the (mu, nu) plane that
 * start and end at x, all with the same orientation:
 *   U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
 *   + U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
 *   + U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
 *   + U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+ .
 * The links are those of the fermion representation.  The improved operator
 * is D_sw = D + A.  `A` receives the 4N x 4N matrix of every site,
 * [V][4N][4N] with row index spin * N + colour.
 */
static void matmul(int n, const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            cplx z = 0;
            for (int k = 0; k < n; k++) z += a[i * n + k] * b[k * n + j];
            c[i * n + j] = z;
        }
}

static void dagger_of(int n, const cplx *a, cplx *c)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) c[i * n + j] = conj(a[j * n + i]);
}

/* product of four matrices a b c d (n x n) */
static void prod4(int n, const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *out)
{
    cplx t1[MAXN * MAXN], t2[MAXN * MAXN];
    matmul(n, a, b, t1);
    matmul(n, t1, c, t2);
    matmul(n, t2, d, out);
}

static const cplx *link_at(const int *d, int n, const cplx *U, int mu, const int x[4])
{
    return U + ((long)mu * volume(d) + lexidx(d, x)) * n * n;
}

static void shifted(const int *d, const int x[4], int mu, int smu, int nu, int snu, int y[4])
{
    memcpy(y, x, 4 * sizeof(int));
    y[mu] = (y[mu] + smu + d[mu]) % d[mu];
    y[nu] = (y[nu] + snu + d[nu]) % d[nu];
}

void oracle_clover(const int *d, int n, const cplx *U, double csw, cplx *A)
{
    const long V = volume(d);
    const int ns = 4 * n;
    cplx G[4][4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        cplx *a = A + s * ns * ns;
        for (int k = 0; k < ns * ns; k++) a[k] = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++) {
                if (mu == nu) continue;
                cplx Q[MAXN * MAXN], L[MAXN * MAXN], d1[MAXN * MAXN], d2[MAXN * MAXN];
                for (int k = 0; k < n * n; k++) Q[k] = 0;
                /* leaf 1 */
                {
                    int y1[4], y2[4];
                    shifted(d, x, mu, 1, nu, 0, y1);
                    shifted(d, x, mu, 0, nu, 1, y2);
                    dagger_of(n, link_at(d, n, U, mu, y2), d1);
                    dagger_of(n, link_at(d, n, U, nu, x), d2);
                    prod4(n, link_at(d, n, U, mu, x), link_at(d, n, U, nu, y1), d1, d2, L);
                    for (int k = 0; k < n * n; k++) Q[k] += L[k];
                }
                /* leaf 2 */
                {
                    int y1[4], y2[4];
                    shifted(d, x, mu, -1, nu, 1, y1);
                    shifted(d, x, mu, -1, nu, 0, y2);
                    cplx d3[MAXN * MAXN];
                    dagger_of(n, link_at(d, n, U, mu, y1), d1);
                    dagger_of(n, link_at(d, n, U, nu, y2), d3);
                    prod4(n, link_at(d, n, U, nu, x), d1, d3, link_at(d, n, U, mu, y2), L);
                    for (int k = 0; k < n * n; k++) Q[k] += L[k];
                }
                /* leaf 3 */
                {
                    int y1[4], y2[4], y3[4];
                    shifted(d, x, mu, -1, nu, 0, y1);
                    shifted(d, x, mu, -1, nu, -1, y2);
                    shifted(d, x, mu, 0, nu, -1, y3);
                    cplx d3[MAXN * MAXN];
                    dagger_of(n, link_at(d, n, U, mu, y1), d1);
                    dagger_of(n, link_at(d, n, U, nu, y2), d3);
                    prod4(n, d1, d3, link_at(d, n, U, mu, y2), link_at(d, n, U, nu, y3), L);
                    for (int k = 0; k < n * n; k++) Q[k] += L[k];
                }
                /* leaf 4 */
                {
                    int y1[4], y2[4];
                    shifted(d, x, mu, 0, nu, -1, y1);
                    shifted(d, x, mu, 1, nu, -1, y2);
                    cplx d3[MAXN * MAXN];
                    dagger_of(n, link_at(d, n, U, nu, y1), d1);
                    dagger_of(n, link_at(d, n, U, mu, x), d3);
                    prod4(n, d1, link_at(d, n, U, mu, y1), link_at(d, n, U, nu, y2), d3, L);
                    for (int k = 0; k < n * n; k++) Q[k] += L[k];
                }
                /* F = (Q - Q^+) / 8 */
                cplx F[MAXN * MAXN];
                for (int i = 0; i < n; i++)
                    for (int j = 0; j < n; j++) F[i * n + j] = (Q[i * n + j] - conj(Q[j * n + i])) / 8.0;
                /* sigma_{mu nu} = (i/2)(g_mu g_nu - g_nu g_mu) */
                cplx sig[4][4];
                for (int a1 = 0; a1 < 4; a1++)
                    for (int b1 = 0; b1 < 4; b1++) {
                        cplx z = 0;
                        for (int k = 0; k < 4; k++) z += G[mu][a1][k] * G[nu][k][b1] - G[nu][a1][k] * G[mu][k][b1];
                        sig[a1][b1] = 0.5 * I * z;
                    }
                /* A += c_sw (i/4) sigma (x) F */
                for (int a1 = 0; a1 < 4; a1++)
                    for (int b1 = 0; b1 < 4; b1++)
                        for (int i = 0; i < n; i++)
                            for (int j = 0; j < n; j++)
                                a[(a1 * n + i) * ns + (b1 * n + j)] += csw * 0.25 * I * sig[a1][b1] * F[i * n + j];
            }
    }
}

/*
 * Conjugate gradients on A = D^+ D^ over the even sites (the same iteration
 * as the Python oracle's cg(), written out in C so that it finishes on the
 * largest lattices):  D^ = m - (1/m) D_eo D_oe with m = 4 + m0 and
 * D_eo = -H_eo / 2 (Sec. 2.1, even/odd preconditioned operator); D^+ =
 * g5 D^ g5 with g5 = g0 g1 g2 g3.  Plain Hestenes-Stiefel from x = 0: stop when
 * the recursively updated ||r|| <= tol ||b||, then recompute b - A x and go on
 * from it if that check fails.  Fields are full-lattice arrays [V][4][n]
 * whose odd sites are ignored on input and zero on output.  Returns the
 * iteration count; *res receives the final ||b - A x|| / ||b||.  With
 * progress > 0 it prints the iterated residual to stderr every `progress`
 * iterations.  Uses
 * 7 temporary full-lattice fields from the heap; returns -1 if they cannot
 * be allocated.
 */
static int site_parity(const int *d, long s)
{
    int x[4];
    coords(d, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* psi <- g5 psi, g5 = g0 g1 g2 g3 formed from the basis above */
static void apply_g5(long V, int n, const cplx *in, cplx *out)
{
    cplx G[4][4][4], t[4][4], g5[4][4];
    for (int mu = 0; mu < 4; mu++) gamma_matrix(mu, G[mu]);
    memcpy(g5, G[0], sizeof(g5));
    for (int mu = 1; mu < 4; mu++) {
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                cplx z = 0;
                for (int k = 0; k < 4; k++) z += g5[a][k] * G[mu][k][b];
                t[a][b] = z;
            }
        memcpy(g5, t, sizeof(g5));
    }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx v[4][MAXN];
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < n; i++) {
                cplx z = 0;
                for (int b = 0; b < 4; b++) z += g5[a][b] * in[(s * 4 + b) * n + i];
                v[a][i] = z;
            }
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < n; i++) out[(s * 4 + a) * n + i] = v[a][i];
    }
}

/* out = D^ in on even sites (zero on odd); tmp: one full-lattice field */
static void dhat_even(const int *d, int n, const cplx *U, const cplx *in, cplx *out, cplx *tmp, double m0)
{
    const long V = volume(d);
    const double m = 4.0 + m0;
    oracle_hopping(d, n, U, in, tmp, 2);  /* H_oe in on odd sites: reads even sites of in only */
#pragma omp parallel for schedule(static)
    for (long k = 0; k < V * 4 * n; k++) tmp[k] *= -0.5; /* D_oe in */
    oracle_hopping(d, n, U, tmp, out, 1); /* H_eo (D_oe in) on even sites */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        const int even = site_parity(d, s) == 0;
        for (long k = s * 4 * n; k < (s + 1) * 4 * n; k++)
            out[k] = even ? m * in[k] - (-0.5 * out[k]) / m : 0;
    }
}

/* out = D^+ D^ in; t1, t2, t3: full-lattice temporaries */
static void normal_even(const int *d, int n, const cplx *U, const cplx *in, cplx *out, cplx *t1, cplx *t2,
                        cplx *t3, double m0)
{
    const long V = volume(d);
    dhat_even(d, n, U, in, t1, t2, m0);
    apply_g5(V, n, t1, t3);
    dhat_even(d, n, U, t3, t1, t2, m0);
    apply_g5(V, n, t1, out);
}

static double re_inner(long N, const cplx *a, const cplx *b)
{
    double s = 0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long k = 0; k < N; k++) s += creal(conj(a[k]) * b[k]);
    return s;
}

int oracle_cg(const int *d, int n, const cplx *U, const cplx *b_in, cplx *x, double m0, double tol, int maxiter,
              double *res, int progress)
{
    const long V = volume(d);
    const long N = V * 4 * n;
    cplx *b = malloc(sizeof(cplx) * N), *r = malloc(sizeof(cplx) * N), *p = malloc(sizeof(cplx) * N);
    cplx *Ap = malloc(sizeof(cplx) * N), *t1 = malloc(sizeof(cplx) * N), *t2 = malloc(sizeof(cplx) * N);
    cplx *t3 = malloc(sizeof(cplx) * N);
    int it = -1;
    if (!b || !r || !p || !Ap || !t1 || !t2 || !t3) goto done;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        const int even = site_parity(d, s) == 0;
        for (long k = s * 4 * n; k < (s + 1) * 4 * n; k++) {
            b[k] = even ? b_in[k] : 0;
            x[k] = 0;
            r[k] = b[k];
            p[k] = b[k];
        }
    }
    const double bnorm = sqrt(re_inner(N, b, b));
    double rr = re_inner(N, r, r);
    it = 0;
    while (it < maxiter) {
        if (sqrt(rr) <= tol * bnorm) {
            normal_even(d, n, U, x, Ap, t1, t2, t3, m0);
#pragma omp parallel for schedule(static)
            for (long k = 0; k < N; k++) t1[k] = b[k] - Ap[k];
            const double rt = re_inner(N, t1, t1);
            if (sqrt(rt) <= tol * bnorm) break;
            memcpy(r, t1, sizeof(cplx) * N);
            memcpy(p, t1, sizeof(cplx) * N);
            rr = rt;
        }
        normal_even(d, n, U, p, Ap, t1, t2, t3, m0);
        const double alpha = rr / re_inner(N, p, Ap);
#pragma omp parallel for schedule(static)
        for (long k = 0; k < N; k++) {
            x[k] += alpha * p[k];
            r[k] -= alpha * Ap[k];
        }
        const double rr_new = re_inner(N, r, r);
        const double beta = rr_new / rr;
#pragma omp parallel for schedule(static)
        for (long k = 0; k < N; k++) p[k] = r[k] + beta * p[k];
        rr = rr_new;
        it++;
        if (progress > 0 && it % progress == 0) {
            fprintf(stderr, "[oracle cg] iteration %d, ||r||/||b|| = %.3e\n", it, sqrt(rr) / bnorm);
            fflush(stderr);
        }
    }
    normal_even(d, n, U, x, Ap, t1, t2, t3, m0);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < N; k++) t1[k] = b[k] - Ap[k];
    *res = sqrt(re_inner(N, t1, t1)) / bnorm;
done:
    free(b), free(r), free(p), free(Ap), free(t1), free(t2), free(t3);
    return it;
}

/* ||b - D^+ D^ x|| / ||b|| over the even sites (odd sites of b and x are
   ignored), with the operator of oracle_cg.  Returns -1 if the temporaries
   cannot be allocated. */
double oracle_true_residual(const int *d, int n, const cplx *U, const cplx *b_in, const cplx *x_in, double m0)
{
    const long V = volume(d);
    const long N = V * 4 * n;
    cplx *b = malloc(sizeof(cplx) * N), *x = malloc(sizeof(cplx) * N), *Ax = malloc(sizeof(cplx) * N);
    cplx *t1 = malloc(sizeof(cplx) * N), *t2 = malloc(sizeof(cplx) * N), *t3 = malloc(sizeof(cplx) * N);
    double res = -1;
    if (b && x && Ax && t1 && t2 && t3) {
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; s++) {
            const int even = site_parity(d, s) == 0;
            for (long k = s * 4 * n; k < (s + 1) * 4 * n; k++) {
                b[k] = even ? b_in[k] : 0;
                x[k] = even ? x_in[k] : 0;
            }
        }
        normal_even(d, n, U, x, Ax, t1, t2, t3, m0);
#pragma omp parallel for schedule(static)
        for (long k = 0; k < N; k++) t1[k] = b[k] - Ax[k];
        res = sqrt(re_inner(N, t1, t1) / re_inner(N, b, b));
    }
    free(b), free(x), free(Ax), free(t1), free(t2), free(t3);
    return res;
}
