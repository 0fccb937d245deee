/*
 * fxo.c -- plain FP64 CPU oracle for the N-body exchange build.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against; it is used by the test-suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark, never by the product path.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What it computes (Challacombe & Bock, "An N-Body Solution to the Problem
 * of Fock Exchange"):
 *   - the exchange contraction of Eq. (6) with the library's scale
 *     convention (factor 1, no -1/2):  K_{mu sig} = sum_{nu lam}
 *     (mu nu|lam sig) P_{nu lam};
 *   - the two-electron integrals over contracted Cartesian Gaussians
 *     (the "standard two-electron integral" the paper cites after Eq. (6)),
 *     here by the McMurchie-Davidson Hermite expansion -- deliberately not
 *     the Head-Gordon-Pople scheme the paper (Section V) and the GPU use;
 *   - the blocked Almlof-Ahlrichs metric query of Eq. (8), evaluated at the
 *     finest block level, single shells: a shell quartet (a,b,c,d) is
 *     computed iff  beta = (Qn_ab * Qn_cd) * Pn_bc > tau  where
 *     Qn_ab = ||(ab|ab)^{1/2}||_F over the functions of the two shells and
 *     Pn_bc = max(||P_bc||_F, ||P_cb||_F).  Because the block Frobenius
 *     norm bounds every sub-block norm, the hextree traversal of Eqs. (7)
 *     computes exactly this quartet set, whatever the tree.
 *
 * Boys function: F_0 from erf for large T, the convergent series
 * F_m(T) = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) for T < 30 and
 * upward recursion F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T) beyond.
 *
 * Every floating-point expression is evaluated as written (build with
 * -ffp-contract=off): the shell-level norms follow a fixed summation order,
 * row-major over the block, so that any other code computing the same
 * definition in the same order obtains bitwise identical norms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXL 2                 /* s, p, d */
#define OMAXL4 (4 * OMAXL)      /* highest total angular momentum */
#define ONC 6                   /* Cartesian components of the highest l */

static const double PI = 3.14159265358979323846264338327950288;

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents of component k of shell l, lexicographic order
 * (x^l first): for l=2 -> xx, xy, xz, yy, yz, zz. */
static void cart_exps(int l, int k, int* ix, int* iy, int* iz) {
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == k) { *ix = i; *iy = j; *iz = l - i - j; return; }
            ++n;
        }
}

static double dfact(int n) { /* (n)!! with (-1)!! = 1 */
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= (double)k;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Boys function                                                             */
/* ------------------------------------------------------------------------ */
void fxo_boys(int mmax, double T, double* F) {
    if (T == 0.0) {
        for (int m = 0; m <= mmax; ++m) F[m] = 1.0 / (2.0 * m + 1.0);
        return;
    }
    double eT = exp(-T);
    if (T < 30.0) {
        for (int m = 0; m <= mmax; ++m) {
            double term = 1.0 / (2.0 * m + 1.0), sum = term;
            for (int k = 1; k < 2000; ++k) {
                term *= 2.0 * T / (2.0 * m + 2.0 * k + 1.0);
                sum += term;
                if (term < 1e-18 * sum) break;
            }
            F[m] = eT * sum;
        }
    } else {
        F[0] = 0.5 * sqrt(PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2.0 * m + 1.0) * F[m] - eT) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------------ */
/* shells                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int l, nprim, f0;
    double A[3];
    const double* alpha;
    double c[ONC][8];   /* per component, per primitive: weight x norm / sqrt(S) */
} oshell;

#define OMAXPRIM 8

/* Normalise: c_p^{ijk} = d_p N_p^{ijk} / sqrt(S^{ijk}) with
 * N^{ijk} = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2i-1)!!(2j-1)!!(2k-1)!!)
 * and S^{ijk} the self-overlap of sum_p d_p N_p^{ijk} g_p^{ijk}. */
static int setup_shells(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                        const double* exps, const double* coefs, oshell* sh) {
    int off = 0, f0 = 0;
    for (int s = 0; s < nshell; ++s) {
        oshell* S = &sh[s];
        if (l[s] < 0 || l[s] > OMAXL || nprim[s] < 1 || nprim[s] > OMAXPRIM) return -1;
        S->l = l[s];
        S->nprim = nprim[s];
        S->f0 = f0;
        S->A[0] = center[3 * s]; S->A[1] = center[3 * s + 1]; S->A[2] = center[3 * s + 2];
        S->alpha = exps + off;
        for (int k = 0; k < ncart(S->l); ++k) {
            int ix = 0, iy = 0, iz = 0;
            cart_exps(S->l, k, &ix, &iy, &iz);
            double df = dfact(2 * ix - 1) * dfact(2 * iy - 1) * dfact(2 * iz - 1);
            double N[OMAXPRIM];
            for (int p = 0; p < S->nprim; ++p) {
                double a = S->alpha[p];
                N[p] = pow(2.0 * a / PI, 0.75) * pow(4.0 * a, 0.5 * S->l) / sqrt(df);
            }
            double ovl = 0.0;
            for (int p = 0; p < S->nprim; ++p)
                for (int q = 0; q < S->nprim; ++q) {
                    double g = S->alpha[p] + S->alpha[q];
                    double prim = df / pow(2.0 * g, S->l) * pow(PI / g, 1.5);
                    ovl += coefs[off + p] * coefs[off + q] * N[p] * N[q] * prim;
                }
            for (int p = 0; p < S->nprim; ++p) S->c[k][p] = coefs[off + p] * N[p] / sqrt(ovl);
        }
        off += S->nprim;
        f0 += ncart(S->l);
    }
    return f0;
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson primitives                                             */
/* ------------------------------------------------------------------------ */
#define ET (2 * OMAXL + 1)
/* E[i][j][t], Hermite expansion coefficients of one Cartesian direction */
static void hermite_E(int la, int lb, double p, double XPA, double XPB, double E00,
                      double E[OMAXL + 1][OMAXL + 1][ET + 1]) {
    memset(E, 0, sizeof(double) * (OMAXL + 1) * (OMAXL + 1) * (ET + 1));
    E[0][0][0] = E00;
    double h = 1.0 / (2.0 * p);
    for (int i = 0; i <= la; ++i) {
        if (i > 0) {
            for (int t = 0; t <= i; ++t) {
                double v = XPA * E[i - 1][0][t];
                if (t > 0) v += h * E[i - 1][0][t - 1];
                if (t + 1 <= i - 1) v += (t + 1) * E[i - 1][0][t + 1];
                E[i][0][t] = v;
            }
        }
        for (int j = 1; j <= lb; ++j) {
            for (int t = 0; t <= i + j; ++t) {
                double v = XPB * E[i][j - 1][t];
                if (t > 0) v += h * E[i][j - 1][t - 1];
                if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                E[i][j][t] = v;
            }
        }
    }
}

#define RD (OMAXL4 + 1)
typedef double rtab[RD][RD][RD][RD]; /* R[n][t][u][v] */

static void hermite_R(int L, double alpha, const double PQ[3], const double* F, rtab R) {
    double m2a = 1.0;
    for (int n = 0; n <= L; ++n) {
        R[n][0][0][0] = m2a * F[n];
        m2a *= -2.0 * alpha;
    }
    for (int s = 1; s <= L; ++s)
        for (int t = 0; t <= s; ++t)
            for (int u = 0; u <= s - t; ++u) {
                int v = s - t - u;
                for (int n = 0; n <= L - s; ++n) {
                    double r;
                    if (t > 0) {
                        r = PQ[0] * R[n + 1][t - 1][u][v];
                        if (t > 1) r += (t - 1) * R[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        r = PQ[1] * R[n + 1][t][u - 1][v];
                        if (u > 1) r += (u - 1) * R[n + 1][t][u - 2][v];
                    } else {
                        r = PQ[2] * R[n + 1][t][u][v - 1];
                        if (v > 1) r += (v - 1) * R[n + 1][t][u][v - 2];
                    }
                    R[n][t][u][v] = r;
                }
            }
}

/* (ab|cd) for one shell quartet, all Cartesian components, accumulated into
 * out[((mu*nb + nu)*nc + lam)*nd + sig].  With diag != 0 (requires c == a
 * and d == b) only the elements (mu nu|mu nu) are formed, into
 * out[mu*nb + nu]. */
static void eri_quartet(const oshell* a, const oshell* b, const oshell* c, const oshell* d,
                        int diag, double* out) {
    int na = ncart(a->l), nb = ncart(b->l), nc = ncart(c->l), nd = ncart(d->l);
    int Lab = a->l + b->l, Lcd = c->l + d->l, L = Lab + Lcd;
    int cab[ONC * ONC][6], ccd[ONC * ONC][6];
    for (int m = 0; m < na; ++m)
        for (int n = 0; n < nb; ++n) {
            int* e = cab[m * nb + n];
            cart_exps(a->l, m, &e[0], &e[1], &e[2]);
            cart_exps(b->l, n, &e[3], &e[4], &e[5]);
        }
    for (int m = 0; m < nc; ++m)
        for (int n = 0; n < nd; ++n) {
            int* e = ccd[m * nd + n];
            cart_exps(c->l, m, &e[0], &e[1], &e[2]);
            cart_exps(d->l, n, &e[3], &e[4], &e[5]);
        }
    int nout = diag ? na * nb : na * nb * nc * nd;
    memset(out, 0, sizeof(double) * nout);

    double AB[3], CD[3];
    for (int x = 0; x < 3; ++x) { AB[x] = a->A[x] - b->A[x]; CD[x] = c->A[x] - d->A[x]; }
    static __thread rtab R;
    double Eab[3][OMAXL + 1][OMAXL + 1][ET + 1], Ecd[3][OMAXL + 1][OMAXL + 1][ET + 1];
    double F[OMAXL4 + 1];
    double G[RD * RD * RD];

    for (int pa = 0; pa < a->nprim; ++pa)
        for (int pb = 0; pb < b->nprim; ++pb) {
            double al = a->alpha[pa], be = b->alpha[pb], p = al + be, mu = al * be / p;
            double P[3];
            for (int x = 0; x < 3; ++x) {
                P[x] = (al * a->A[x] + be * b->A[x]) / p;
                hermite_E(a->l, b->l, p, P[x] - a->A[x], P[x] - b->A[x], exp(-mu * AB[x] * AB[x]), Eab[x]);
            }
            for (int pc = 0; pc < c->nprim; ++pc)
                for (int pd = 0; pd < d->nprim; ++pd) {
                    double ga = c->alpha[pc], de = d->alpha[pd], q = ga + de, nu = ga * de / q;
                    double Q[3], PQ[3];
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (ga * c->A[x] + de * d->A[x]) / q;
                        hermite_E(c->l, d->l, q, Q[x] - c->A[x], Q[x] - d->A[x], exp(-nu * CD[x] * CD[x]), Ecd[x]);
                        PQ[x] = P[x] - Q[x];
                    }
                    double alpha = p * q / (p + q);
                    double T = alpha * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
                    fxo_boys(L, T, F);
                    hermite_R(L, alpha, PQ, F, R);
                    double pref = 2.0 * pow(PI, 2.5) / (p * q * sqrt(p + q));
                    int cd_n = diag ? 1 : nc * nd;
                    for (int cdi = 0; cdi < (diag ? na * nb : cd_n); ++cdi) {
                        /* ket component pair; in diag mode it equals the bra pair */
                        int cd = cdi;
                        const int* f = ccd[cd];
                        int la_ = cd / nd, si_ = cd % nd;
                        /* G_{tuv} = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi} */
                        for (int t = 0; t <= Lab; ++t)
                            for (int u = 0; u <= Lab - t; ++u)
                                for (int v = 0; v <= Lab - t - u; ++v) {
                                    double g = 0.0;
                                    for (int tt = 0; tt <= f[0] + f[3]; ++tt)
                                        for (int uu = 0; uu <= f[1] + f[4]; ++uu)
                                            for (int vv = 0; vv <= f[2] + f[5]; ++vv) {
                                                double ecd = Ecd[0][f[0]][f[3]][tt] * Ecd[1][f[1]][f[4]][uu] *
                                                             Ecd[2][f[2]][f[5]][vv];
                                                double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                                                g += sg * ecd * R[0][t + tt][u + uu][v + vv];
                                            }
                                    G[(t * RD + u) * RD + v] = g;
                                }
                        int ab_lo = diag ? cdi : 0, ab_hi = diag ? cdi + 1 : na * nb;
                        for (int ab = ab_lo; ab < ab_hi; ++ab) {
                            const int* e = cab[ab];
                            int mu_ = ab / nb, nu_ = ab % nb;
                            double w = pref * a->c[mu_][pa] * b->c[nu_][pb] * c->c[la_][pc] * d->c[si_][pd];
                            /* sum_{tuv} E^{ab}_{tuv} G_{tuv} */
                            double acc = 0.0;
                            for (int t = 0; t <= e[0] + e[3]; ++t)
                                for (int u = 0; u <= e[1] + e[4]; ++u)
                                    for (int v = 0; v <= e[2] + e[5]; ++v)
                                        acc += Eab[0][e[0]][e[3]][t] * Eab[1][e[1]][e[4]][u] *
                                               Eab[2][e[2]][e[5]][v] * G[(t * RD + u) * RD + v];
                            if (diag) out[ab] += w * acc;
                            else out[ab * nc * nd + cd] += w * acc;
                        }
                    }
                }
        }
    (void)Lcd;
}

/* ------------------------------------------------------------------------ */
/* public entry points                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nshell, nbf;
    oshell* sh;
} obasis;

static int make_basis(obasis* B, int nshell, const int32_t* l, const int32_t* nprim,
                      const double* center, const double* exps, const double* coefs) {
    B->nshell = nshell;
    B->sh = (oshell*)calloc((size_t)nshell, sizeof(oshell));
    if (!B->sh) return -1;
    B->nbf = setup_shells(nshell, l, nprim, center, exps, coefs, B->sh);
    if (B->nbf < 0) { free(B->sh); return -1; }
    return 0;
}

/* Normalised contraction weights, c[(shell*6 + comp)*8 + prim]. */
int fxo_norm_coefs(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                   const double* exps, const double* coefs, double* c_out) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    for (int s = 0; s < nshell; ++s)
        for (int k = 0; k < ONC; ++k)
            for (int p = 0; p < OMAXPRIM; ++p) c_out[(s * ONC + k) * OMAXPRIM + p] = B.sh[s].c[k][p];
    free(B.sh);
    return 0;
}

/* All Cartesian integrals of one shell quartet. */
int fxo_eri_quartet(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                    const double* exps, const double* coefs, int a, int b, int c, int d, double* out) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    eri_quartet(&B.sh[a], &B.sh[b], &B.sh[c], &B.sh[d], 0, out);
    free(B.sh);
    return 0;
}

/* Full four-index tensor (n^4 doubles), every quartet, no screening. */
int fxo_eri_tensor(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                   const double* exps, const double* coefs, double* T) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int n = B.nbf, S = nshell;
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < S; ++a) {
        double buf[ONC * ONC * ONC * ONC];
        for (int b = 0; b < S; ++b)
            for (int c = 0; c < S; ++c)
                for (int d = 0; d < S; ++d) {
                    const oshell *A = &B.sh[a], *Bb = &B.sh[b], *C = &B.sh[c], *D = &B.sh[d];
                    eri_quartet(A, Bb, C, D, 0, buf);
                    int na = ncart(A->l), nb = ncart(Bb->l), nc = ncart(C->l), nd = ncart(D->l);
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int m = 0; m < nd; ++m)
                                    T[(((size_t)(A->f0 + i) * n + (Bb->f0 + j)) * n + (C->f0 + k)) * n + (D->f0 + m)] =
                                        buf[((i * nb + j) * nc + k) * nd + m];
                }
    }
    free(B.sh);
    return 0;
}

static void schwarz_norms(const obasis* B, double* Qn) {
    int S = B->nshell;
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < S; ++a) {
        double buf[ONC * ONC];
        for (int b = a; b < S; ++b) {
            const oshell *A = &B->sh[a], *Bb = &B->sh[b];
            /* skip pairs whose Gaussian-product prefactors all underflow:
             * the diagonal integral is then below 1e-250 */
            double r2 = 0.0;
            for (int x = 0; x < 3; ++x) r2 += (A->A[x] - Bb->A[x]) * (A->A[x] - Bb->A[x]);
            double emin = 1e300;
            for (int p = 0; p < A->nprim; ++p)
                for (int q = 0; q < Bb->nprim; ++q) {
                    double e = A->alpha[p] * Bb->alpha[q] / (A->alpha[p] + Bb->alpha[q]) * r2;
                    if (e < emin) emin = e;
                }
            double s2 = 0.0;
            if (emin < 575.0) {
                eri_quartet(A, Bb, A, Bb, 1, buf);
                int nab = ncart(A->l) * ncart(Bb->l);
                for (int k = 0; k < nab; ++k) s2 += buf[k] > 0.0 ? buf[k] : 0.0;
            }
            double v = sqrt(s2);
            Qn[(size_t)a * S + b] = v;
            Qn[(size_t)b * S + a] = v;
        }
    }
}

/* Qn[a*S+b] = ||Q_ab||_F with Q_{mu nu} = sqrt(max(0, (mu nu|mu nu))). */
int fxo_schwarz(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                const double* exps, const double* coefs, double* Qn) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    schwarz_norms(&B, Qn);
    free(B.sh);
    return 0;
}

/* ||P_bc||_F summed row-major over the block (mu outer, nu inner). */
static double block_frob(const double* P, int n, int r0, int nr, int c0, int ncol) {
    double s = 0.0;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < ncol; ++j) {
            double v = P[(size_t)(r0 + i) * n + (c0 + j)];
            s += v * v;
        }
    return sqrt(s);
}

/* Pn[b*S+c] = max(||P_bc||_F, ||P_cb||_F). */
int fxo_pnorm(int nshell, const int32_t* l, const double* P, double* Pn) {
    int* f0 = (int*)malloc(sizeof(int) * (nshell + 1));
    f0[0] = 0;
    for (int s = 0; s < nshell; ++s) f0[s + 1] = f0[s] + ncart(l[s]);
    int n = f0[nshell];
#pragma omp parallel for schedule(static)
    for (int b = 0; b < nshell; ++b)
        for (int c = b; c < nshell; ++c) {
            double x = block_frob(P, n, f0[b], f0[b + 1] - f0[b], f0[c], f0[c + 1] - f0[c]);
            double y = block_frob(P, n, f0[c], f0[c + 1] - f0[c], f0[b], f0[b + 1] - f0[b]);
            double v = x > y ? x : y;
            Pn[(size_t)b * nshell + c] = v;
            Pn[(size_t)c * nshell + b] = v;
        }
    free(f0);
    return 0;
}

/* contract one quartet into a K block: Kblk[mu*ldk + sig] += sum (mu nu|lam sig) P_{nu lam} */
static void contract(const oshell* A, const oshell* Bb, const oshell* C, const oshell* D, const double* I,
                     const double* P, int n, double* Krow, int ldk, int kcol0) {
    int na = ncart(A->l), nb = ncart(Bb->l), nc = ncart(C->l), nd = ncart(D->l);
    for (int i = 0; i < na; ++i)
        for (int m = 0; m < nd; ++m) {
            double s = 0.0;
            for (int j = 0; j < nb; ++j)
                for (int k = 0; k < nc; ++k)
                    s += I[((i * nb + j) * nc + k) * nd + m] * P[(size_t)(Bb->f0 + j) * n + (C->f0 + k)];
            Krow[(size_t)i * ldk + kcol0 + m] += s;
        }
}

typedef struct { double q; int idx; } qi;
static int cmp_qi_desc(const void* x, const void* y) {
    const qi* a = (const qi*)x; const qi* b = (const qi*)y;
    if (a->q > b->q) return -1;
    if (a->q < b->q) return 1;
    return a->idx - b->idx;
}

/* Per c: shells d sorted by descending Qn[c][d]. */
static int* sorted_partners(const double* Qn, int S) {
    int* ord = (int*)malloc(sizeof(int) * (size_t)S * S);
    qi* tmp = (qi*)malloc(sizeof(qi) * (size_t)S * S);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < S; ++c) {
        qi* t = tmp + (size_t)c * S;
        for (int d = 0; d < S; ++d) { t[d].q = Qn[(size_t)c * S + d]; t[d].idx = d; }
        qsort(t, S, sizeof(qi), cmp_qi_desc);
        for (int d = 0; d < S; ++d) ord[(size_t)c * S + d] = t[d].idx;
    }
    free(tmp);
    return ord;
}

/*
 * Screened exchange.  K (n x n, row-major, overwritten) receives
 *   K_{mu sig} = sum over shell quartets with beta > tau of
 *                sum_{nu in b, lam in c} (mu nu|lam sig) P_{nu lam}.
 * tau < 0 computes every quartet (brute force).
 * Qn/Pn may be NULL (computed here) or caller-provided shell norms.
 * stats (nullable): [0] computed quartets, [1] quartets with
 * |beta/tau - 1| < 1e-10 (threshold-sensitive), [2] primitive quartets.
 */
int fxo_exchange(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                 const double* exps, const double* coefs, const double* P, double tau,
                 double* K, double* stats) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int S = nshell, n = B.nbf;
    double* Qn = (double*)malloc(sizeof(double) * (size_t)S * S);
    double* Pn = (double*)malloc(sizeof(double) * (size_t)S * S);
    schwarz_norms(&B, Qn);
    fxo_pnorm(S, l, P, Pn);
    int* ord = sorted_partners(Qn, S);
    double qmax = 0.0, pmax = 0.0;
    for (size_t i = 0; i < (size_t)S * S; ++i) {
        if (Qn[i] > qmax) qmax = Qn[i];
        if (Pn[i] > pmax) pmax = Pn[i];
    }
    memset(K, 0, sizeof(double) * (size_t)n * n);
    double nq = 0, nnear = 0, nprimq = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : nq, nnear, nprimq)
    for (int a = 0; a < S; ++a) {
        const oshell* A = &B.sh[a];
        double* Krow = K + (size_t)A->f0 * n;   /* rows of shell a: owned by this iteration */
        double buf[ONC * ONC * ONC * ONC];
        for (int b = 0; b < S; ++b) {
            double qab = Qn[(size_t)a * S + b];
            if (tau >= 0.0 && (qab * qmax) * pmax <= tau) continue;
            for (int c = 0; c < S; ++c) {
                double pbc = Pn[(size_t)b * S + c];
                const int* dl = ord + (size_t)c * S;
                for (int k = 0; k < S; ++k) {
                    int d = dl[k];
                    double beta = (qab * Qn[(size_t)c * S + d]) * pbc;
                    if (tau >= 0.0 && !(beta > tau)) break;
                    if (tau > 0.0 && fabs(beta / tau - 1.0) < 1e-10) nnear += 1;
                    const oshell *Bb = &B.sh[b], *C = &B.sh[c], *D = &B.sh[d];
                    eri_quartet(A, Bb, C, D, 0, buf);
                    contract(A, Bb, C, D, buf, P, n, Krow, n, D->f0);
                    nq += 1;
                    nprimq += (double)A->nprim * Bb->nprim * C->nprim * D->nprim;
                }
            }
        }
    }
    if (stats) { stats[0] = nq; stats[1] = nnear; stats[2] = nprimq; }
    free(ord); free(Qn); free(Pn); free(B.sh);
    return 0;
}

/*
 * Screened exchange through the permutational symmetry of the integrals
 * (Section IV, Eqs. 9-10).  Every unique shell quartet is taken once, in the
 * canonical order a >= b, c >= d, ab >= cd (pair index ab = a(a+1)/2 + b),
 * its integrals are evaluated once, and they are contracted into the K block
 * of every distinct ordered quartet they stand for -- (ab|cd), (ba|cd),
 * (ab|dc), (ba|dc) and the four with the two pairs exchanged, an integral
 * (pq|rs) adding (pq|rs) P_qr to K_ps -- each kept under its own bound
 * beta = (Qn_pq Qn_rs) Pn_qr > tau, as fxo_exchange keeps it.  The result is
 * therefore fxo_exchange's K up to the order of the sums, while the
 * integral evaluations drop to about an eighth.  tau < 0: every quartet.
 * Serial: the contributions of one integral land in up to eight K blocks.
 * stats (nullable): [0] unique quartets whose integrals were evaluated,
 * [1] ordered quartets contracted (fxo_exchange's computed count), [2]
 * primitive quartets of the evaluated integrals, and a shell-level analogue
 * of the paper's breakdown by symmetry block (its Fig. 2): of the evaluated
 * quartets, [3] those with eight distinct images all kept (the full 4-fold
 * contraction of Eq. 9 on both pairs), [4] those with coinciding indices
 * (fewer distinct images, all kept: the diagonal cases), [5] those with
 * some distinct image culled by its own bound (the "sparse" cases).
 */
int fxo_exchange_sym8(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                      const double* exps, const double* coefs, const double* P, double tau, double* K,
                      double* stats) {
    static const int perm[8][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
                                   {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int S = nshell, n = B.nbf;
    double* Qn = (double*)malloc(sizeof(double) * (size_t)S * S);
    double* Pn = (double*)malloc(sizeof(double) * (size_t)S * S);
    schwarz_norms(&B, Qn);
    fxo_pnorm(S, l, P, Pn);
    memset(K, 0, sizeof(double) * (size_t)n * n);
    double nint = 0, nq = 0, nprimq = 0, nfull = 0, ndiag = 0, nsparse = 0;
    double buf[ONC * ONC * ONC * ONC];
    for (int a = 0; a < S; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= a; ++c)
                for (int d = 0; d <= c; ++d) {
                    if (c * (c + 1) / 2 + d > a * (a + 1) / 2 + b) continue;
                    const int sh[4] = {a, b, c, d};
                    /* the distinct images (p,q,r,s), the slot map of each (pidx) and
                       whether its own bound keeps it */
                    int img[8][4], pidx[8], keep[8], nimg = 0, any = 0;
                    for (int x = 0; x < 8; ++x) {
                        int t[4];
                        for (int y = 0; y < 4; ++y) t[y] = sh[perm[x][y]];
                        int dup = 0;
                        for (int z = 0; z < nimg && !dup; ++z)
                            dup = img[z][0] == t[0] && img[z][1] == t[1] && img[z][2] == t[2] && img[z][3] == t[3];
                        if (dup) continue;
                        memcpy(img[nimg], t, sizeof(t));
                        const double beta = (Qn[(size_t)t[0] * S + t[1]] * Qn[(size_t)t[2] * S + t[3]]) *
                                            Pn[(size_t)t[1] * S + t[2]];
                        pidx[nimg] = x;
                        keep[nimg] = tau < 0.0 || beta > tau;
                        any |= keep[nimg];
                        ++nimg;
                    }
                    if (!any) continue;
                    int nkeep = 0;
                    for (int z = 0; z < nimg; ++z) nkeep += keep[z];
                    if (nkeep < nimg) nsparse += 1;
                    else if (nimg == 8) nfull += 1;
                    else ndiag += 1;
                    const oshell* Sh[4] = {&B.sh[a], &B.sh[b], &B.sh[c], &B.sh[d]};
                    eri_quartet(Sh[0], Sh[1], Sh[2], Sh[3], 0, buf);
                    nint += 1;
                    nprimq += (double)Sh[0]->nprim * Sh[1]->nprim * Sh[2]->nprim * Sh[3]->nprim;
                    const int nc4[4] = {ncart(Sh[0]->l), ncart(Sh[1]->l), ncart(Sh[2]->l), ncart(Sh[3]->l)};
                    for (int z = 0; z < nimg; ++z) {
                        if (!keep[z]) continue;
                        const int* pm = perm[pidx[z]];
                        const oshell *Ps = Sh[pm[0]], *Qs = Sh[pm[1]], *Rs = Sh[pm[2]], *Ss = Sh[pm[3]];
                        const int np_ = nc4[pm[0]], nq_ = nc4[pm[1]], nr_ = nc4[pm[2]], ns_ = nc4[pm[3]];
                        for (int i = 0; i < np_; ++i)
                            for (int m = 0; m < ns_; ++m) {
                                double acc = 0.0;
                                for (int j = 0; j < nq_; ++j)
                                    for (int k = 0; k < nr_; ++k) {
                                        int t[4];
                                        t[pm[0]] = i; t[pm[1]] = j; t[pm[2]] = k; t[pm[3]] = m;
                                        const double I = buf[((t[0] * nc4[1] + t[1]) * nc4[2] + t[2]) * nc4[3] + t[3]];
                                        acc += I * P[(size_t)(Qs->f0 + j) * n + (Rs->f0 + k)];
                                    }
                                K[(size_t)(Ps->f0 + i) * n + (Ss->f0 + m)] += acc;
                            }
                        nq += 1;
                    }
                }
    if (stats) {
        stats[0] = nint; stats[1] = nq; stats[2] = nprimq;
        stats[3] = nfull; stats[4] = ndiag; stats[5] = nsparse;
    }
    free(Qn); free(Pn); free(B.sh);
    return 0;
}

/*
 * Overlap integrals (phi_mu|phi_nu) of the normalised contracted functions,
 * by the Hermite expansion: a Gaussian product in one direction is
 * sum_t E_t^{ij} Lambda_t, and only the t = 0 Hermite function has a
 * non-zero integral, sqrt(pi/p); so (mu|nu) = sum_pq c c E_0^x E_0^y E_0^z
 * (pi/p)^{3/2} (the E00 factors carry exp(-a b / p X_AB^2) per direction).
 * Smax[a*S+b] = max over mu in a, nu in b of |(mu|nu)|: the quantity the
 * overlap criterion of Eqs. (3)-(4) compares with tau_ovlp.  S (n x n,
 * nullable) receives the full overlap matrix.
 */
static void shell_overlap(const oshell* A, const oshell* B, double* blk) {
    int na = ncart(A->l), nb = ncart(B->l);
    memset(blk, 0, sizeof(double) * na * nb);
    double E[3][OMAXL + 1][OMAXL + 1][ET + 1];
    for (int p = 0; p < A->nprim; ++p)
        for (int q = 0; q < B->nprim; ++q) {
            double a = A->alpha[p], b = B->alpha[q], g = a + b;
            for (int x = 0; x < 3; ++x) {
                double P = (a * A->A[x] + b * B->A[x]) / g, X = A->A[x] - B->A[x];
                hermite_E(A->l, B->l, g, P - A->A[x], P - B->A[x], exp(-a * b / g * X * X), E[x]);
            }
            double pre = pow(PI / g, 1.5);
            for (int i = 0; i < na; ++i) {
                int ix = 0, iy = 0, iz = 0;
                cart_exps(A->l, i, &ix, &iy, &iz);
                for (int j = 0; j < nb; ++j) {
                    int jx = 0, jy = 0, jz = 0;
                    cart_exps(B->l, j, &jx, &jy, &jz);
                    blk[i * nb + j] += A->c[i][p] * B->c[j][q] * E[0][ix][jx][0] * E[1][iy][jy][0] *
                                       E[2][iz][jz][0] * pre;
                }
            }
        }
}

int fxo_overlap(int nshell, const int32_t* l, const int32_t* nprim, const double* center, const double* exps,
                const double* coefs, double* Smax, double* S) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int NS = nshell, n = B.nbf;
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < NS; ++a) {
        double blk[ONC * ONC];
        for (int b = 0; b < NS; ++b) {
            const oshell *A = &B.sh[a], *Bb = &B.sh[b];
            shell_overlap(A, Bb, blk);
            double m = 0.0;
            int na = ncart(A->l), nb = ncart(Bb->l);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    double v = fabs(blk[i * nb + j]);
                    if (v > m) m = v;
                    if (S) S[(size_t)(A->f0 + i) * n + Bb->f0 + j] = blk[i * nb + j];
                }
            Smax[(size_t)a * NS + b] = m;
        }
    }
    free(B.sh);
    return 0;
}

/*
 * Screened exchange with the overlap criterion of Eqs. (3)-(4) as well: a
 * shell pair whose largest overlap is below tau_ovlp contributes nothing,
 * so a quartet (a,b,c,d) is computed iff beta > tau and Smax_ab >= tau_ovlp
 * and Smax_cd >= tau_ovlp.  tau_ovlp = 0 gives fxo_exchange.  stats as in
 * fxo_exchange, plus [3] quartets that beta alone would keep.
 */
int fxo_exchange_ovlp(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                      const double* exps, const double* coefs, const double* P, double tau, double tau_ovlp,
                      double* K, double* stats) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int S = nshell, n = B.nbf;
    double* Qn = (double*)malloc(sizeof(double) * (size_t)S * S);
    double* Pn = (double*)malloc(sizeof(double) * (size_t)S * S);
    double* Sm = (double*)malloc(sizeof(double) * (size_t)S * S);
    schwarz_norms(&B, Qn);
    fxo_pnorm(S, l, P, Pn);
    fxo_overlap(nshell, l, nprim, center, exps, coefs, Sm, NULL);
    memset(K, 0, sizeof(double) * (size_t)n * n);
    double nq = 0, nnear = 0, nbeta = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : nq, nnear, nbeta)
    for (int a = 0; a < S; ++a) {
        const oshell* A = &B.sh[a];
        double* Krow = K + (size_t)A->f0 * n;
        double buf[ONC * ONC * ONC * ONC];
        for (int b = 0; b < S; ++b)
            for (int c = 0; c < S; ++c)
                for (int d = 0; d < S; ++d) {
                    double beta = (Qn[(size_t)a * S + b] * Qn[(size_t)c * S + d]) * Pn[(size_t)b * S + c];
                    if (!(beta > tau)) continue;
                    nbeta += 1;
                    if (tau > 0.0 && fabs(beta / tau - 1.0) < 1e-10) nnear += 1;
                    double sab = Sm[(size_t)a * S + b], scd = Sm[(size_t)c * S + d];
                    if (tau_ovlp > 0.0 && (fabs(sab / tau_ovlp - 1.0) < 1e-10 || fabs(scd / tau_ovlp - 1.0) < 1e-10))
                        nnear += 1;
                    if (!(sab >= tau_ovlp) || !(scd >= tau_ovlp)) continue;
                    const oshell *Bb = &B.sh[b], *C = &B.sh[c], *D = &B.sh[d];
                    eri_quartet(A, Bb, C, D, 0, buf);
                    contract(A, Bb, C, D, buf, P, n, Krow, n, D->f0);
                    nq += 1;
                }
    }
    if (stats) { stats[0] = nq; stats[1] = nnear; stats[2] = 0; stats[3] = nbeta; }
    free(Qn); free(Pn); free(Sm); free(B.sh);
    return 0;
}

/*
 * The paper's leaf rule (Section V: the recursion ends at blocks of at most
 * ten functions, which are evaluated whole).  The basis, in the given shell
 * order, is bisected as in Eq. (1): a block of shells is split at the shell
 * boundary nearest its function midpoint (the lower one on a tie) until it
 * holds at most leaf_max functions or a single shell.  A leaf task
 * (A,B,C,D) is kept iff its block bound of Eq. (8), in squared norms,
 *     (Qsq_AB * Qsq_CD) * Psq_BC * (1 + 1e-12) > tau^2,
 * with Qsq_AB the sum of Qn_ab^2 over the shell pairs of the two blocks
 * (a ascending, then b) and Psq likewise from Pn.  Every shell quartet of a
 * kept task is computed, whatever its own bound.  The block norms of the
 * enclosing tasks are no smaller, so the leaf test alone decides.
 * stats (nullable): [0] computed quartets, [1] leaf tasks whose bound lies
 * within 1e-10 relative of the threshold, [2] kept leaf tasks, [3] leaves.
 */
static int leaf_split(const int* fp, int lo, int hi, int leaf_max, int* lo_out, int nl) {
    if (fp[hi] - fp[lo] <= leaf_max || hi - lo == 1) {
        lo_out[nl] = lo;
        return nl + 1;
    }
    double mid = 0.5 * (double)(fp[lo] + fp[hi]);
    int best = lo + 1;
    double bd = 1e300;
    for (int m = lo + 1; m < hi; ++m) {
        double dd = fabs((double)fp[m] - mid);
        if (dd < bd) { bd = dd; best = m; }
    }
    nl = leaf_split(fp, lo, best, leaf_max, lo_out, nl);
    return leaf_split(fp, best, hi, leaf_max, lo_out, nl);
}

int fxo_exchange_leafblock(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                           const double* exps, const double* coefs, const double* P, double tau, int leaf_max,
                           double* K, double* stats) {
    obasis B;
    if (leaf_max < 1) return -1;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int S = nshell, n = B.nbf;
    double* Qn = (double*)malloc(sizeof(double) * (size_t)S * S);
    double* Pn = (double*)malloc(sizeof(double) * (size_t)S * S);
    schwarz_norms(&B, Qn);
    fxo_pnorm(S, l, P, Pn);
    int* fp = (int*)malloc(sizeof(int) * (S + 1));
    fp[0] = 0;
    for (int s = 0; s < S; ++s) fp[s + 1] = fp[s] + ncart(l[s]);
    int* lo = (int*)malloc(sizeof(int) * (S + 1));
    int NL = leaf_split(fp, 0, S, leaf_max, lo, 0);
    lo[NL] = S;
    double* Qsq = (double*)malloc(sizeof(double) * (size_t)NL * NL);
    double* Psq = (double*)malloc(sizeof(double) * (size_t)NL * NL);
    for (int X = 0; X < NL; ++X)
        for (int Y = 0; Y < NL; ++Y) {
            double q = 0.0, pp = 0.0;
            for (int a = lo[X]; a < lo[X + 1]; ++a)
                for (int b = lo[Y]; b < lo[Y + 1]; ++b) {
                    double v = Qn[(size_t)a * S + b], w = Pn[(size_t)a * S + b];
                    q += v * v;
                    pp += w * w;
                }
            Qsq[(size_t)X * NL + Y] = q;
            Psq[(size_t)X * NL + Y] = pp;
        }
    memset(K, 0, sizeof(double) * (size_t)n * n);
    const double tau2 = tau * tau;
    double nq = 0, nnear = 0, nkept = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : nq, nnear, nkept)
    for (int A = 0; A < NL; ++A) {
        double buf[ONC * ONC * ONC * ONC];
        for (int D = 0; D < NL; ++D)
            for (int Bk = 0; Bk < NL; ++Bk)
                for (int C = 0; C < NL; ++C) {
                    double b2 = (Qsq[(size_t)A * NL + Bk] * Qsq[(size_t)C * NL + D]) * Psq[(size_t)Bk * NL + C];
                    double t = b2 * (1.0 + 1e-12);
                    if (tau > 0.0 && fabs(t / tau2 - 1.0) < 1e-10) nnear += 1;
                    if (!(t > tau2)) continue;
                    nkept += 1;
                    for (int a = lo[A]; a < lo[A + 1]; ++a)
                        for (int d = lo[D]; d < lo[D + 1]; ++d)
                            for (int b = lo[Bk]; b < lo[Bk + 1]; ++b)
                                for (int c = lo[C]; c < lo[C + 1]; ++c) {
                                    const oshell *Sa = &B.sh[a], *Sb = &B.sh[b], *Sc = &B.sh[c], *Sd = &B.sh[d];
                                    eri_quartet(Sa, Sb, Sc, Sd, 0, buf);
                                    contract(Sa, Sb, Sc, Sd, buf, P, n, K + (size_t)Sa->f0 * n, n, Sd->f0);
                                    nq += 1;
                                }
                }
    }
    if (stats) { stats[0] = nq; stats[1] = nnear; stats[2] = nkept; stats[3] = NL; }
    free(Qsq); free(Psq); free(lo); free(fp); free(Qn); free(Pn); free(B.sh);
    return 0;
}

/*
 * Sampled K blocks: for each requested shell pair (a,d) the na x nd block
 * of the screened K, out concatenated block after block (row-major each).
 * Qn/Pn: caller-provided shell norms (from fxo_schwarz / fxo_pnorm).
 */
int fxo_exchange_blocks(int nshell, const int32_t* l, const int32_t* nprim, const double* center,
                        const double* exps, const double* coefs, const double* P, double tau,
                        const double* Qn, const double* Pn, int npairs, const int32_t* pairs,
                        double* out, double* stats) {
    obasis B;
    if (make_basis(&B, nshell, l, nprim, center, exps, coefs)) return -1;
    int S = nshell, n = B.nbf;
    size_t* off = (size_t*)malloc(sizeof(size_t) * (npairs + 1));
    off[0] = 0;
    for (int i = 0; i < npairs; ++i)
        off[i + 1] = off[i] + (size_t)ncart(B.sh[pairs[2 * i]].l) * ncart(B.sh[pairs[2 * i + 1]].l);
    memset(out, 0, sizeof(double) * off[npairs]);
    double nq = 0, nnear = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : nq, nnear)
    for (int i = 0; i < npairs; ++i) {
        int a = pairs[2 * i], d = pairs[2 * i + 1];
        const oshell *A = &B.sh[a], *D = &B.sh[d];
        double buf[ONC * ONC * ONC * ONC];
        int nd = ncart(D->l);
        for (int b = 0; b < S; ++b)
            for (int c = 0; c < S; ++c) {
                double beta = (Qn[(size_t)a * S + b] * Qn[(size_t)c * S + d]) * Pn[(size_t)b * S + c];
                if (tau >= 0.0 && !(beta > tau)) continue;
                if (tau > 0.0 && fabs(beta / tau - 1.0) < 1e-10) nnear += 1;
                eri_quartet(A, &B.sh[b], &B.sh[c], D, 0, buf);
                contract(A, &B.sh[b], &B.sh[c], D, buf, P, n, out + off[i], nd, 0);
                nq += 1;
            }
    }
    if (stats) { stats[0] = nq; stats[1] = nnear; }
    free(off); free(B.sh);
    return 0;
}

/*
 * Bound matrix of the culled work: E_{mu sig} = sum over culled quartets
 * (a,b,c,d) with mu in a, sig in d of beta.  By Cauchy-Schwarz and
 * |(mu nu|lam sig)| <= Q_{mu nu} Q_{lam sig}, the contribution a culled
 * quartet would have made to K_{mu sig} is at most its beta, so
 * |K_tau - K_full| <= E elementwise.  Exhaustive: tiny systems only.
 */
int fxo_bound_matrix(int nshell, const int32_t* l, const double* Qn, const double* Pn, double tau,
                     double* E) {
    int S = nshell;
    int* f0 = (int*)malloc(sizeof(int) * (S + 1));
    f0[0] = 0;
    for (int s = 0; s < S; ++s) f0[s + 1] = f0[s] + ncart(l[s]);
    int n = f0[S];
    memset(E, 0, sizeof(double) * (size_t)n * n);
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < S; ++a)
        for (int d = 0; d < S; ++d) {
            double e = 0.0;
            for (int b = 0; b < S; ++b)
                for (int c = 0; c < S; ++c) {
                    double beta = (Qn[(size_t)a * S + b] * Qn[(size_t)c * S + d]) * Pn[(size_t)b * S + c];
                    if (!(beta > tau)) e += beta;
                }
            for (int i = f0[a]; i < f0[a + 1]; ++i)
                for (int j = f0[d]; j < f0[d + 1]; ++j) E[(size_t)i * n + j] = e;
        }
    free(f0);
    return 0;
}

/*
 * Exact count of surviving ordered shell quartets, per angular-momentum
 * class (counts[((la*3+lb)*3+lc)*3+ld]), plus the primitive-quartet total
 * and the number of threshold-sensitive quartets (|beta/tau-1| < 1e-10).
 * Same enumeration and test as fxo_exchange, without the integrals.
 */
int fxo_count(int nshell, const int32_t* l, const int32_t* nprim, const double* Qn, const double* Pn,
              double tau, double* counts, double* prim_total, double* near_total) {
    int S = nshell;
    int* ord = sorted_partners(Qn, S);
    double qmax = 0.0, pmax = 0.0;
    for (size_t i = 0; i < (size_t)S * S; ++i) {
        if (Qn[i] > qmax) qmax = Qn[i];
        if (Pn[i] > pmax) pmax = Pn[i];
    }
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double* part = (double*)calloc((size_t)nthr * 81, sizeof(double));
    double np = 0, nn = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : np, nn)
    for (int a = 0; a < S; ++a) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* cnt = part + (size_t)tid * 81;
        for (int b = 0; b < S; ++b) {
            double qab = Qn[(size_t)a * S + b];
            if ((qab * qmax) * pmax <= tau) continue;
            for (int c = 0; c < S; ++c) {
                double pbc = Pn[(size_t)b * S + c];
                const int* dl = ord + (size_t)c * S;
                for (int k = 0; k < S; ++k) {
                    int d = dl[k];
                    double beta = (qab * Qn[(size_t)c * S + d]) * pbc;
                    if (!(beta > tau)) break;
                    if (tau > 0.0 && fabs(beta / tau - 1.0) < 1e-10) nn += 1;
                    cnt[((l[a] * 3 + l[b]) * 3 + l[c]) * 3 + l[d]] += 1;
                    np += (double)nprim[a] * nprim[b] * nprim[c] * nprim[d];
                }
            }
        }
    }
    for (int k = 0; k < 81; ++k) {
        counts[k] = 0;
        for (int t = 0; t < nthr; ++t) counts[k] += part[(size_t)t * 81 + k];
    }
    *prim_total = np;
    *near_total = nn;
    free(part); free(ord);
    return 0;
}

/* Threads the oracle's parallel loops use (OpenMP); n < 1 leaves it unchanged. */
void fxo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int fxo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
