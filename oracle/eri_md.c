/*
 * Two-electron repulsion integrals over Cartesian Gaussian primitives by the
 * McMurchie-Davidson scheme, and the Boys function.
 *
 * TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle.  It serves the
 * brute-force deterministic MP2 energy (the four-index transformation of
 * Sec. II, Eq. transformation, feeding Eq. FinalMP2) on tiny inputs.
 *
 * Primitive: N (x-Ax)^lx (y-Ay)^ly (z-Az)^lz exp(-a |r-A|^2).
 *
 * Hermite expansion of a 1D overlap distribution (exponents a, b, centres
 * A, B; p = a + b, P = (aA + bB)/p):
 *   E^{00}_0 = exp(-ab/p (A-B)^2),
 *   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + (P-A) E^{ij}_t + (t+1) E^{ij}_{t+1},
 *   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + (P-B) E^{ij}_t + (t+1) E^{ij}_{t+1}.
 * Hermite Coulomb integrals (alpha = pq/(p+q), X = P-Q, T = alpha |P-Q|^2):
 *   R^n_{000} = (-2 alpha)^n F_n(T),
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_x R^{n+1}_{t,u,v}   (same for u, v).
 * ERI:
 *   (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q))
 *             sum_{tuv} E^{ab}_{tuv} sum_{t'u'v'} (-1)^{t'+u'+v'} E^{cd}_{t'u'v'} R^0_{t+t',u+u',v+v'}.
 * Boys function F_n(T) = int_0^1 t^{2n} exp(-T t^2) dt: series
 *   F_n(T) = exp(-T) sum_k (2T)^k / ((2n+1)(2n+3)...(2n+2k+1))
 * at the highest order and downward recursion F_{n-1} = (2T F_n + exp(-T))/(2n-1)
 * for T < 40; above, F_0 = sqrt(pi/T) erf(sqrt T)/2 and upward recursion.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LMAX 4                 /* per primitive */
#define LT (4 * LMAX)          /* total in an integral */
#define NE (2 * LMAX + 1)      /* Hermite index range of a pair */

void oracle_boys(int nmax, double T, double *F) {
    if (T < 40.0) {
        double term = 1.0 / (2 * nmax + 1), sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= 2.0 * T / (2 * nmax + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        double eT = exp(-T);
        F[nmax] = eT * sum;
        for (int n = nmax; n > 0; --n) F[n - 1] = (2.0 * T * F[n] + eT) / (2 * n - 1);
    } else {
        double eT = exp(-T);
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int n = 0; n < nmax; ++n) F[n + 1] = ((2 * n + 1) * F[n] - eT) / (2.0 * T);
    }
}

/* E[i][j][t], i <= la, j <= lb, t <= i + j; 1D. */
static void hermite_e(int la, int lb, double a, double b, double A, double B,
                      double E[LMAX + 1][LMAX + 1][NE + 1]) {
    double p = a + b, P = (a * A + b * B) / p;
    double XPA = P - A, XPB = P - B, h = 0.5 / p;
    memset(E, 0, sizeof(double) * (LMAX + 1) * (LMAX + 1) * (NE + 1));
    E[0][0][0] = exp(-a * b / p * (A - B) * (A - B));
    for (int i = 0; i <= la; ++i) {
        for (int j = 0; j <= lb; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (i > 0) {
                    v = XPA * E[i - 1][j][t];
                    if (t > 0) v += h * E[i - 1][j][t - 1];
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                } else {
                    v = XPB * E[i][j - 1][t];
                    if (t > 0) v += h * E[i][j - 1][t - 1];
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                }
                E[i][j][t] = v;
            }
        }
    }
}

/* R[t][u][v] = R^0_{tuv}, t+u+v <= L. */
static void hermite_r(int L, double alpha, double X, double Y, double Z,
                      double R[LT + 1][LT + 1][LT + 1]) {
    static double Rn[LT + 1][LT + 1][LT + 1][LT + 1];
    double F[LT + 1];
    double T = alpha * (X * X + Y * Y + Z * Z);
    oracle_boys(L, T, F);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) {
        Rn[n][0][0][0] = f * F[n];
        f *= -2.0 * alpha;
    }
    /* build levels of increasing t+u+v; R^n needs R^{n+1} of the lower level */
    for (int s = 1; s <= L; ++s) {
        for (int n = 0; n <= L - s; ++n) {
            for (int t = 0; t <= s; ++t) {
                for (int u = 0; u <= s - t; ++u) {
                    int v = s - t - u;
                    double val;
                    if (t > 0) {
                        val = X * Rn[n + 1][t - 1][u][v];
                        if (t > 1) val += (t - 1) * Rn[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        val = Y * Rn[n + 1][t][u - 1][v];
                        if (u > 1) val += (u - 1) * Rn[n + 1][t][u - 2][v];
                    } else {
                        val = Z * Rn[n + 1][t][u][v - 1];
                        if (v > 1) val += (v - 1) * Rn[n + 1][t][u][v - 2];
                    }
                    Rn[n][t][u][v] = val;
                }
            }
        }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) R[t][u][v] = Rn[0][t][u][v];
}

typedef struct {
    double p, P[3];
    int l[3];                           /* la + lb per axis */
    double E[3][NE + 1];                /* E^{ab}_t per axis */
    double pref;                        /* product of norms */
} pairdata;

static void make_pair(const double *xyz, const double *alpha, const int *lxyz, const double *norm,
                      int i, int j, pairdata *pd) {
    static double E[LMAX + 1][LMAX + 1][NE + 1];
    double a = alpha[i], b = alpha[j];
    pd->p = a + b;
    for (int d = 0; d < 3; ++d) {
        int la = lxyz[3 * i + d], lb = lxyz[3 * j + d];
        hermite_e(la, lb, a, b, xyz[3 * i + d], xyz[3 * j + d], E);
        pd->P[d] = (a * xyz[3 * i + d] + b * xyz[3 * j + d]) / pd->p;
        pd->l[d] = la + lb;
        for (int t = 0; t <= NE; ++t) pd->E[d][t] = (t <= la + lb) ? E[la][lb][t] : 0.0;
    }
    pd->pref = norm[i] * norm[j];
}

static double eri_pairpair(const pairdata *ab, const pairdata *cd) {
    static double R[LT + 1][LT + 1][LT + 1];
    double p = ab->p, q = cd->p, alpha = p * q / (p + q);
    int L = ab->l[0] + ab->l[1] + ab->l[2] + cd->l[0] + cd->l[1] + cd->l[2];
    hermite_r(L, alpha, ab->P[0] - cd->P[0], ab->P[1] - cd->P[1], ab->P[2] - cd->P[2], R);
    double sum = 0.0;
    for (int t = 0; t <= ab->l[0]; ++t)
        for (int u = 0; u <= ab->l[1]; ++u)
            for (int v = 0; v <= ab->l[2]; ++v) {
                double eab = ab->E[0][t] * ab->E[1][u] * ab->E[2][v];
                if (eab == 0.0) continue;
                double inner = 0.0;
                for (int t2 = 0; t2 <= cd->l[0]; ++t2)
                    for (int u2 = 0; u2 <= cd->l[1]; ++u2)
                        for (int v2 = 0; v2 <= cd->l[2]; ++v2) {
                            double ecd = cd->E[0][t2] * cd->E[1][u2] * cd->E[2][v2];
                            double sgn = ((t2 + u2 + v2) & 1) ? -1.0 : 1.0;
                            inner += sgn * ecd * R[t + t2][u + u2][v + v2];
                        }
                sum += eab * inner;
            }
    return 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * sum * ab->pref * cd->pref;
}

/*
 * (ij|kl) for every pair of the npairs charge distributions listed in
 * (pi[n], pj[n]): out[P * npairs + Q] = (pi[P] pj[P] | pi[Q] pj[Q]).
 * Returns 0, or -1 if a primitive exceeds LMAX or allocation fails.
 */
int oracle_eri_pairs(int nprim, const double *xyz, const double *alpha, const int *lxyz,
                     const double *norm, int npairs, const int *pi, const int *pj, double *out) {
    for (int i = 0; i < nprim; ++i)
        if (lxyz[3 * i] + lxyz[3 * i + 1] + lxyz[3 * i + 2] > LMAX) return -1;
    pairdata *pd = (pairdata *)malloc(sizeof(pairdata) * (size_t)(npairs > 0 ? npairs : 1));
    if (!pd) return -1;
    for (int P = 0; P < npairs; ++P) make_pair(xyz, alpha, lxyz, norm, pi[P], pj[P], &pd[P]);
    for (int P = 0; P < npairs; ++P)
        for (int Q = 0; Q <= P; ++Q) {
            double v = eri_pairpair(&pd[P], &pd[Q]);
            out[(size_t)P * npairs + Q] = v;
            out[(size_t)Q * npairs + P] = v;
        }
    free(pd);
    return 0;
}
