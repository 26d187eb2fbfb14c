/*
 * Oracle for the RPA polarizability hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference in complex128 (pairs of
 * doubles, real part first).  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark call this code; the product path
 * never does.  It shares no code, header or table with the GPU library.
 *
 * Every function computes a plain definition from the paper:
 *   orc_pair_density  plane-wave matrix element (matrix-element equation of
 *                     the epsilon section) evaluated exactly in the
 *                     plane-wave basis: a convolution over G-vectors.
 *   orc_weights       energy denominators of the static-chi equation and
 *                     its imaginary-frequency continuation.
 *   orc_weights_real  the complex retarded/advanced weights at real
 *                     frequencies (full-frequency epsilon).
 *   orc_chi_cw        the chi sum with those complex weights.
 *   orc_ff_grid       the real-frequency grid of the full-frequency run.
 *   orc_chi           the chi sum itself, for every (G, G') asked for,
 *                     with compensated summation over the pair index.
 *   orc_vcoul         bare Coulomb interaction of the untruncated bulk case.
 *   orc_eps           dielectric matrix, asymmetric-Coulomb form.
 *   orc_inverse       Gaussian elimination with partial pivoting on [A | I]
 *                     (the ZGESV semantics the paper names for the
 *                     inversion), LAPACK INFO convention.
 *   orc_realify       real coefficients from complex ones (real flavor):
 *                     Gram-Schmidt over the real and imaginary parts of
 *                     each degenerate group of states.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HARTREE_EV 27.211386245988 /* CODATA 2018, eV per hartree */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Neumaier-compensated accumulation: s is the running sum, c the carry. */
static inline void neu_add(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static int max_abs_component(int n, const int *g)
{
    int r = 0;
    for (int i = 0; i < 3 * n; ++i) {
        int a = g[i] < 0 ? -g[i] : g[i];
        if (a > r) r = a;
    }
    return r;
}

/*
 * Plane-wave matrix element (epsilon section, matrix-element equation):
 *   M_t(G) = <v,k+q| e^{i(q+G).r} |c,k>
 *          = sum_{G2 in wfn sphere, G+G2 in wfn sphere} conj(Cv(G+G2)) Cc(G2)
 * with psi_nk = V^{-1/2} sum_G C_nk(G) e^{i(k+G).r}; the Bloch phases cancel.
 * Pair index t = (k*nv + v)*nc + c.  cv: [nk][nv][ngw] (valence at k+q),
 * cc: [nk][nc][ngw] (conduction at k).  Output M: [npairs][ng], for the pair
 * indices listed in `pairs` (all K pairs in order when pairs == NULL).
 * The sum over G2 runs in ascending wavefunction-sphere order.
 */
int orc_pair_density(int ngw, const int *gw, int ng, const int *ge,
                     int nk, int nv, int nc, const double *cv, const double *cc,
                     long npairs, const long *pairs, double *M)
{
    if (ngw <= 0 || ng <= 0 || nk <= 0 || nv <= 0 || nc <= 0) return -1;
    const long K = (long)nk * nv * nc;
    if (pairs == NULL) npairs = K;
    const int rw = max_abs_component(ngw, gw), re = max_abs_component(ng, ge);
    const int off = rw + re, side = 2 * off + 1;
    const long boxn = (long)side * side * side;
    int *box = (int *)malloc(sizeof(int) * boxn);
    if (!box) return -5;
    for (long i = 0; i < boxn; ++i) box[i] = -1;
    for (int i = 0; i < ngw; ++i) {
        long p = ((long)(gw[3 * i] + off) * side + (gw[3 * i + 1] + off)) * side + (gw[3 * i + 2] + off);
        box[p] = i;
    }
    /* index of ge[g] + gw[g2] in the wavefunction sphere, or -1 */
    int *sum_idx = (int *)malloc(sizeof(int) * (size_t)ng * ngw);
    if (!sum_idx) { free(box); return -5; }
#pragma omp parallel for schedule(static)
    for (int g = 0; g < ng; ++g)
        for (int g2 = 0; g2 < ngw; ++g2) {
            int x = ge[3 * g] + gw[3 * g2] + off;
            int y = ge[3 * g + 1] + gw[3 * g2 + 1] + off;
            int z = ge[3 * g + 2] + gw[3 * g2 + 2] + off;
            sum_idx[(size_t)g * ngw + g2] = box[((long)x * side + y) * side + z];
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (long p = 0; p < npairs; ++p) {
        long t = pairs ? pairs[p] : p;
        long c = t % nc, kv = t / nc;          /* kv = k*nv + v */
        long k = kv / nv;
        const double *a = cv + 2 * kv * ngw;
        const double *b = cc + 2 * (k * nc + c) * ngw;
        double *out = M + 2 * p * ng;
        for (int g = 0; g < ng; ++g) {
            const int *idx = sum_idx + (size_t)g * ngw;
            double sr = 0, cr = 0, si = 0, ci = 0;
            for (int g2 = 0; g2 < ngw; ++g2) {
                int j = idx[g2];
                if (j < 0) continue;
                double ar = a[2 * j], ai = a[2 * j + 1];
                double br = b[2 * g2], bi = b[2 * g2 + 1];
                /* conj(a) * b */
                neu_add(&sr, &cr, ar * br + ai * bi);
                neu_add(&si, &ci, ar * bi - ai * br);
            }
            out[2 * g] = sr + cr;
            out[2 * g + 1] = si + ci;
        }
    }
    free(sum_idx);
    free(box);
    return 0;
}

/*
 * Energy weights.  Static-chi equation: 1/(E_{v,k+q} - E_{c,k}); the
 * imaginary-frequency reading evaluates the retarded form at E = i*omega,
 * delta -> 0+, which gives Delta/(Delta^2 + omega^2) (real, negative).
 * Energies and omega in eV, converted to hartree.  w: [nw][K].
 */
int orc_weights(int nk, int nv, int nc, const double *ev, const double *ec,
                int nw, const double *omega_ev, double *w)
{
    if (nk <= 0 || nv <= 0 || nc <= 0 || nw <= 0) return -1;
    const long K = (long)nk * nv * nc;
    for (int iw = 0; iw < nw; ++iw) {
        if (omega_ev[iw] < 0) return -1;
        double om = omega_ev[iw] / HARTREE_EV;
        for (long t = 0; t < K; ++t) {
            long c = t % nc, kv = t / nc, k = kv / nv, v = kv % nv;
            double d = (ev[k * nv + v] - ec[k * nc + c]) / HARTREE_EV;
            w[iw * K + t] = d / (d * d + om * om);
        }
    }
    return 0;
}

/*
 * Real-frequency weights of the retarded/advanced dielectric equation
 * (full-frequency part of the epsilon section):
 *   w_t(E) = 1/2 [ 1/(Delta_t - E - i s delta) + 1/(Delta_t + E + i s delta) ]
 * with s = +1 for the retarded function and s = -1 for the advanced one,
 * Delta_t = E_{v,k+q} - E_{c,k}; every input in eV, converted to hartree.
 * Complex division written out: 1/(x + i y) = (x - i y)/(x^2 + y^2).
 * w: [nE][K] complex (re, im interleaved).
 */
int orc_weights_real(int nk, int nv, int nc, const double *ev, const double *ec,
                     int nE, const double *E_ev, double delta_ev, int retarded, double *w)
{
    if (nk <= 0 || nv <= 0 || nc <= 0 || nE <= 0 || !(delta_ev > 0)) return -1;
    const long K = (long)nk * nv * nc;
    const double s = retarded ? 1.0 : -1.0;
    const double dl = s * delta_ev / HARTREE_EV;
    for (int ie = 0; ie < nE; ++ie) {
        if (E_ev[ie] < 0) return -1;
        double E = E_ev[ie] / HARTREE_EV;
        for (long t = 0; t < K; ++t) {
            long c = t % nc, kv = t / nc, k = kv / nv, v = kv % nv;
            double d = (ev[k * nv + v] - ec[k * nc + c]) / HARTREE_EV;
            /* first term: 1/(x1 + i y1), x1 = d - E, y1 = -dl */
            double x1 = d - E, y1 = -dl, n1 = x1 * x1 + y1 * y1;
            /* second term: 1/(x2 + i y2), x2 = d + E, y2 = +dl */
            double x2 = d + E, y2 = dl, n2 = x2 * x2 + y2 * y2;
            w[2 * (ie * K + t)] = 0.5 * (x1 / n1 + x2 / n2);
            w[2 * (ie * K + t) + 1] = 0.5 * (-y1 / n1 - y2 / n2);
        }
    }
    return 0;
}

/*
 * The chi sum with complex weights (real frequency axis): every requested
 * entry chi_{GG'}(E) = pf * sum_t conj(M_t(G)) w_t(E) M_t(G'), summed over t
 * in ascending order with Neumaier compensation.  w: [nE][K] complex.
 * rows/cols as in orc_chi.
 */
int orc_chi_cw(long K, int ng, const double *M, int nw, const double *w, double pf,
               int nrow, const int *rows, int ncol, const int *cols, double *chi)
{
    if (K < 0 || ng <= 0 || nw <= 0) return -1;
    if (!rows) nrow = ng;
    if (!cols) ncol = ng;
    for (int iw = 0; iw < nw; ++iw) {
        const double *wv = w + 2L * iw * K;
#pragma omp parallel
        {
            double *acc = (double *)malloc(sizeof(double) * 4 * ncol);
#pragma omp for schedule(dynamic, 1)
            for (int r = 0; r < nrow; ++r) {
                int g = rows ? rows[r] : r;
                memset(acc, 0, sizeof(double) * 4 * ncol);
                for (long t = 0; t < K; ++t) {
                    const double *mt = M + 2 * t * ng;
                    /* a = w_t * conj(M_t(G)) */
                    double cr = mt[2 * g], ci = -mt[2 * g + 1];
                    double wr = wv[2 * t], wi = wv[2 * t + 1];
                    double ar = wr * cr - wi * ci, ai = wr * ci + wi * cr;
                    for (int cidx = 0; cidx < ncol; ++cidx) {
                        int g2 = cols ? cols[cidx] : cidx;
                        double br = mt[2 * g2], bi = mt[2 * g2 + 1];
                        double *s = acc + 4 * cidx;
                        neu_add(&s[0], &s[1], ar * br - ai * bi);
                        neu_add(&s[2], &s[3], ar * bi + ai * br);
                    }
                }
                double *out = chi + 2 * ((long)iw * nrow * ncol + (long)r * ncol);
                for (int cidx = 0; cidx < ncol; ++cidx) {
                    out[2 * cidx] = pf * (acc[4 * cidx] + acc[4 * cidx + 1]);
                    out[2 * cidx + 1] = pf * (acc[4 * cidx + 2] + acc[4 * cidx + 3]);
                }
            }
            free(acc);
        }
    }
    return 0;
}

/*
 * Real-frequency grid of the full-frequency epsilon calculation (the paper's
 * frequency-grid figure): uniform from 0 with spacing dE up to the low
 * cutoff, then the spacing grows by `increment` at every further point until
 * the high cutoff.  Writes at most maxn points to E (eV) and returns the
 * number of points the grid has (which may exceed maxn), or -1.
 */
int orc_ff_grid(double dE, double e_low, double e_high, double increment, int maxn, double *E)
{
    if (!(dE > 0) || e_low < 0 || e_high < e_low || increment < 0) return -1;
    int n = 0;
    double x = 0.0;
    /* uniform part: i * dE for i = 0, 1, ... while <= e_low */
    for (long i = 0;; ++i) {
        x = (double)i * dE;
        if (x > e_low * (1.0 + 1e-12)) break;
        if (n < maxn) E[n] = x;
        ++n;
    }
    x = (double)(n - 1) * dE;
    double step = dE;
    for (;;) {
        step += increment;
        double next = x + step;
        if (next > e_high * (1.0 + 1e-12)) break;
        if (n < maxn) E[n] = next;
        ++n;
        x = next;
        if (increment == 0 && n > 10000000) return -1;
    }
    return n;
}

/*
 * chi_{GG'}(omega) = pf * sum_t conj(M_t(G)) w_t(omega) M_t(G')   (static-chi
 * equation, with the implicit 1/(N_k V_uc) normalisation passed in as pf).
 * Every requested entry is summed independently over t in ascending order
 * with Neumaier compensation.  rows/cols select G and G' (NULL = all ng).
 * M: [K][ng]; w: [nw][K]; chi: [nw][nrow][ncol].
 */
int orc_chi(long K, int ng, const double *M, int nw, const double *w, double pf,
            int nrow, const int *rows, int ncol, const int *cols, double *chi)
{
    if (K < 0 || ng <= 0 || nw <= 0) return -1;
    if (!rows) nrow = ng;
    if (!cols) ncol = ng;
    for (int iw = 0; iw < nw; ++iw) {
        const double *wv = w + (long)iw * K;
#pragma omp parallel
        {
            double *acc = (double *)malloc(sizeof(double) * 4 * ncol);
#pragma omp for schedule(dynamic, 1)
            for (int r = 0; r < nrow; ++r) {
                int g = rows ? rows[r] : r;
                memset(acc, 0, sizeof(double) * 4 * ncol);
                for (long t = 0; t < K; ++t) {
                    const double *mt = M + 2 * t * ng;
                    double ar = mt[2 * g] * wv[t], ai = -mt[2 * g + 1] * wv[t]; /* w * conj(M_t(G)) */
                    for (int cidx = 0; cidx < ncol; ++cidx) {
                        int g2 = cols ? cols[cidx] : cidx;
                        double br = mt[2 * g2], bi = mt[2 * g2 + 1];
                        double *s = acc + 4 * cidx;
                        neu_add(&s[0], &s[1], ar * br - ai * bi);
                        neu_add(&s[2], &s[3], ar * bi + ai * br);
                    }
                }
                double *out = chi + 2 * ((long)iw * nrow * ncol + (long)r * ncol);
                for (int cidx = 0; cidx < ncol; ++cidx) {
                    out[2 * cidx] = pf * (acc[4 * cidx] + acc[4 * cidx + 1]);
                    out[2 * cidx + 1] = pf * (acc[4 * cidx + 2] + acc[4 * cidx + 3]);
                }
            }
            free(acc);
        }
    }
    return 0;
}

/*
 * Bulk bare Coulomb interaction v(q+G) = 4 pi / |q+G|^2.
 * bvec: reciprocal lattice vectors as rows (bohr^-1), q in crystal units,
 * ge: Miller triples.  Returns -3 if some |q+G| is zero.
 */
/*
 * Exchange kernel of the Bethe-Salpeter equation (optical-properties
 * section, exchange-term equation): for pairs t = (k, v, c) and t',
 *     Kx[t][t'] = pf * sum over G != G0 of conj(M_t(G)) v(q+G) M_t'(G),
 * the G = 0 term (index `head`, or none when head < 0) left out.  Rows
 * `rows` (all if NULL) of the K x K result; compensated summation over G.
 */
int orc_bse_kx(long K, int ng, const double *M, const double *v, int head, double pf,
               int nrow, const long *rows, double *kx)
{
    if (K <= 0 || ng <= 0) return -1;
    if (!rows) nrow = (int)K;
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * 4 * K);
#pragma omp for schedule(dynamic, 1)
        for (int r = 0; r < nrow; ++r) {
            long t = rows ? rows[r] : r;
            const double *mt = M + 2 * t * ng;
            memset(acc, 0, sizeof(double) * 4 * K);
            for (int g = 0; g < ng; ++g) {
                if (g == head) continue;
                double ar = mt[2 * g] * v[g], ai = -mt[2 * g + 1] * v[g]; /* v(G) conj(M_t(G)) */
                for (long t2 = 0; t2 < K; ++t2) {
                    double br = M[2 * (t2 * ng + g)], bi = M[2 * (t2 * ng + g) + 1];
                    double *s = acc + 4 * t2;
                    neu_add(&s[0], &s[1], ar * br - ai * bi);
                    neu_add(&s[2], &s[3], ar * bi + ai * br);
                }
            }
            double *out = kx + 2 * (long)r * K;
            for (long t2 = 0; t2 < K; ++t2) {
                out[2 * t2] = pf * (acc[4 * t2] + acc[4 * t2 + 1]);
                out[2 * t2 + 1] = pf * (acc[4 * t2 + 2] + acc[4 * t2 + 3]);
            }
        }
        free(acc);
    }
    return 0;
}

/*
 * Static self-energy matrix elements of one q (self-energy section): with
 * M[i][n][G] = M_{n''n}(G) for inner states i = n'' and outer states n,
 *   kind 0, bare exchange (hf-x equation):
 *     S[n][n'] = -pf sum_i sum_{G != head} conj(M[i][n][G]) v(G) M[i][n'][G]
 *   kind 1, screened exchange (cohsex-sx equation):
 *     S[n][n'] = -pf sum_i sum_{G,G'} conj(M[i][n][G]) einv[G][G'] v(G') M[i][n'][G']
 *   kind 2, Coulomb hole, sum form (cohsex-ch-sum equation):
 *     S[n][n'] = pf/2 sum_i sum_{G,G'} conj(M[i][n][G]) (einv[G][G'] - delta) v(G') M[i][n'][G']
 * (the inner states summed over are the occupied ones for kinds 0 and 1 and
 * all of them for kind 2: the caller passes that set).  Compensated sums.
 */
int orc_sigma(int kind, int ninner, int nouter, int ng, const double *M, int head, const double *v,
              const double *einv, double pf, double *S)
{
    if (ninner <= 0 || nouter <= 0 || ng <= 0 || kind < 0 || kind > 2) return -1;
    if (kind > 0 && !einv) return -1;
    const double scale = kind == 2 ? 0.5 * pf : -pf;
#pragma omp parallel
    {
        double *y = (double *)malloc(sizeof(double) * 2 * ng);
        double *acc = (double *)malloc(sizeof(double) * 4 * nouter);
#pragma omp for schedule(dynamic, 1)
        for (int n = 0; n < nouter; ++n) {
            memset(acc, 0, sizeof(double) * 4 * nouter);
            for (int i = 0; i < ninner; ++i) {
                const double *mn = M + 2 * ((long)i * nouter + n) * ng;
                /* y[G'] = sum_G conj(M[i][n][G]) Weff[G][G'] (a row vector) */
                for (int g2 = 0; g2 < ng; ++g2) {
                    double yr = 0.0, yi = 0.0;
                    if (kind == 0) {
                        if (g2 != head) {
                            yr = mn[2 * g2] * v[g2];
                            yi = -mn[2 * g2 + 1] * v[g2];
                        }
                    } else {
                        double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
                        for (int g = 0; g < ng; ++g) {
                            double er = einv[2 * ((long)g * ng + g2)], ei = einv[2 * ((long)g * ng + g2) + 1];
                            if (kind == 2 && g == g2) er -= 1.0;
                            double ar = mn[2 * g], ai = -mn[2 * g + 1]; /* conj(M) */
                            neu_add(&sr, &cr, ar * er - ai * ei);
                            neu_add(&si, &ci, ar * ei + ai * er);
                        }
                        yr = (sr + cr) * v[g2];
                        yi = (si + ci) * v[g2];
                    }
                    y[2 * g2] = yr;
                    y[2 * g2 + 1] = yi;
                }
                for (int n2 = 0; n2 < nouter; ++n2) {
                    const double *mm = M + 2 * ((long)i * nouter + n2) * ng;
                    double *s = acc + 4 * n2;
                    for (int g2 = 0; g2 < ng; ++g2) {
                        double br = mm[2 * g2], bi = mm[2 * g2 + 1];
                        neu_add(&s[0], &s[1], y[2 * g2] * br - y[2 * g2 + 1] * bi);
                        neu_add(&s[2], &s[3], y[2 * g2] * bi + y[2 * g2 + 1] * br);
                    }
                }
            }
            double *out = S + 2 * (long)n * nouter;
            for (int n2 = 0; n2 < nouter; ++n2) {
                out[2 * n2] = scale * (acc[4 * n2] + acc[4 * n2 + 1]);
                out[2 * n2 + 1] = scale * (acc[4 * n2 + 2] + acc[4 * n2 + 3]);
            }
        }
        free(acc);
        free(y);
    }
    return 0;
}

int orc_vcoul(const double *bvec, const double *q, int ng, const int *ge, double *v)
{
    for (int g = 0; g < ng; ++g) {
        double m[3] = {q[0] + ge[3 * g], q[1] + ge[3 * g + 1], q[2] + ge[3 * g + 2]};
        double x[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 3; ++d) x[d] += m[i] * bvec[3 * i + d];
        double q2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        if (q2 == 0.0) return -3;
        v[g] = 4.0 * M_PI / q2;
    }
    return 0;
}

/* epsilon_{GG'} = delta_{GG'} - v(q+G) chi_{GG'} ; chi, eps: [nw][ng][ng]. */
int orc_eps(int ng, int nw, const double *v, const double *chi, double *eps)
{
    for (long iw = 0; iw < nw; ++iw)
        for (long g = 0; g < ng; ++g)
            for (long h = 0; h < ng; ++h) {
                long i = 2 * ((iw * ng + g) * ng + h);
                eps[i] = (g == h ? 1.0 : 0.0) - v[g] * chi[i];
                eps[i + 1] = -v[g] * chi[i + 1];
            }
    return 0;
}

/*
 * Inverse by Gaussian elimination with partial pivoting on the augmented
 * system [A | I] (solve A X = I).  Pivot: first row of largest |Re|+|Im|
 * in the current column.  Returns 0, or i > 0 when the i-th pivot
 * (1-based) is exactly zero; Ainv is then left unspecified.
 * A, Ainv: [n][n] complex, row-major.
 */
int orc_inverse(int n, const double *A, double *Ainv)
{
    const long w = 2L * n; /* augmented width in complex entries */
    /* BGW_ORACLE_PROGRESS set: one line on stderr every 512 rows (long runs) */
    const int progress = getenv("BGW_ORACLE_PROGRESS") != NULL;
    double *T = (double *)malloc(sizeof(double) * 2 * (size_t)n * w);
    if (!T) return -5;
    for (long i = 0; i < n; ++i) {
        for (long j = 0; j < n; ++j) {
            T[2 * (i * w + j)] = A[2 * (i * n + j)];
            T[2 * (i * w + j) + 1] = A[2 * (i * n + j) + 1];
            T[2 * (i * w + n + j)] = (i == j) ? 1.0 : 0.0;
            T[2 * (i * w + n + j) + 1] = 0.0;
        }
    }
    int info = 0;
    for (long k = 0; k < n && !info; ++k) {
        if (progress && k % 512 == 0) {
            fprintf(stderr, "[oracle] inverse n=%d: elimination row %ld\n", n, k);
            fflush(stderr);
        }
        long p = k;
        double best = fabs(T[2 * (k * w + k)]) + fabs(T[2 * (k * w + k) + 1]);
        for (long i = k + 1; i < n; ++i) {
            double a = fabs(T[2 * (i * w + k)]) + fabs(T[2 * (i * w + k) + 1]);
            if (a > best) { best = a; p = i; }
        }
        if (best == 0.0) { info = (int)k + 1; break; }
        if (p != k)
            for (long j = 0; j < w; ++j) {
                double t0 = T[2 * (k * w + j)], t1 = T[2 * (k * w + j) + 1];
                T[2 * (k * w + j)] = T[2 * (p * w + j)];
                T[2 * (k * w + j) + 1] = T[2 * (p * w + j) + 1];
                T[2 * (p * w + j)] = t0;
                T[2 * (p * w + j) + 1] = t1;
            }
        double pr = T[2 * (k * w + k)], pi = T[2 * (k * w + k) + 1];
#pragma omp parallel for schedule(static)
        for (long i = k + 1; i < n; ++i) {
            /* l = T[i][k] / pivot */
            double ar = T[2 * (i * w + k)], ai = T[2 * (i * w + k) + 1];
            double den = pr * pr + pi * pi;
            double lr = (ar * pr + ai * pi) / den, li = (ai * pr - ar * pi) / den;
            T[2 * (i * w + k)] = 0.0;
            T[2 * (i * w + k) + 1] = 0.0;
            for (long j = k + 1; j < w; ++j) {
                double br = T[2 * (k * w + j)], bi = T[2 * (k * w + j) + 1];
                T[2 * (i * w + j)] -= lr * br - li * bi;
                T[2 * (i * w + j) + 1] -= lr * bi + li * br;
            }
        }
    }
    if (!info) {
        /* back substitution, all n right-hand sides at once (row-oriented:
         * X[k][:] = (B[k][:] - sum_{m>k} U[k][m] X[m][:]) / U[k][k]) */
        for (long k = n - 1; k >= 0; --k) {
            if (progress && k % 512 == 0) {
                fprintf(stderr, "[oracle] inverse n=%d: back substitution row %ld\n", n, k);
                fflush(stderr);
            }
            double pr = T[2 * (k * w + k)], pi = T[2 * (k * w + k) + 1];
            double den = pr * pr + pi * pi;
#pragma omp parallel for schedule(static)
            for (long jb = n; jb < w; jb += 32) {
                long je = jb + 32 < w ? jb + 32 : w;
                double *xk = T + 2 * k * w;
                for (long m = k + 1; m < n; ++m) {
                    double ur = xk[2 * m], ui = xk[2 * m + 1];
                    const double *xm = T + 2 * m * w;
                    for (long j = jb; j < je; ++j) {
                        xk[2 * j] -= ur * xm[2 * j] - ui * xm[2 * j + 1];
                        xk[2 * j + 1] -= ur * xm[2 * j + 1] + ui * xm[2 * j];
                    }
                }
                for (long j = jb; j < je; ++j) {
                    double sr = xk[2 * j], si = xk[2 * j + 1];
                    xk[2 * j] = (sr * pr + si * pi) / den;
                    xk[2 * j + 1] = (si * pr - sr * pi) / den;
                }
            }
        }
        for (long i = 0; i < n; ++i)
            memcpy(Ainv + 2 * i * n, T + 2 * (i * w + n), sizeof(double) * 2 * n);
    }
    free(T);
    return info;
}

/*
 * Real coefficients from complex ones (the real and complex flavors): with
 * inversion and time-reversal symmetry every state can be chosen with real
 * plane-wave coefficients.  A non-degenerate state is real times a global
 * phase; a group of d degenerate states spans d real dimensions.  Bands of
 * one k are grouped by degeneracy (consecutive bands whose energies differ
 * by at most tol from their neighbour).  For each group the 2d real vectors
 * Re c_b, Im c_b (b in the group, in that order) go through Gram-Schmidt:
 * at each of d steps the remaining vector of largest norm is taken (lowest
 * index on ties), normalised, written as the next real state of the group,
 * and projected out of the remaining vectors.  For one state this divides
 * out its phase (up to sign).
 * c: complex128 [nk][nb][ngw]; e: [nk][nb] (ascending per k); r: real
 * [nk][nb][ngw] out.  Returns the number of groups whose vectors span more
 * than d real dimensions (a remaining norm above 1e-6 after the d steps:
 * the input was not real up to a unitary within the group) or that span
 * fewer, or -1 on bad arguments.
 */
int orc_realify(int nk, int nb, int ngw, const double *c, const double *e, double tol, double *r)
{
    if (nk < 1 || nb < 1 || ngw < 1 || !(tol >= 0.0) || !c || !e || !r) return -1;
    double *v = malloc(sizeof(double) * 2 * (size_t)nb * ngw);
    char *used = malloc((size_t)2 * nb);
    if (!v || !used) {
        free(v);
        free(used);
        return -1;
    }
    int bad = 0;
    for (int k = 0; k < nk; ++k) {
        const double *ek = e + (size_t)k * nb;
        int b0 = 0;
        while (b0 < nb) {
            int b1 = b0 + 1;
            while (b1 < nb && ek[b1] - ek[b1 - 1] <= tol) ++b1;
            const int d = b1 - b0, m = 2 * d;
            for (int i = 0; i < d; ++i) {
                const double *cb = c + 2 * ((size_t)k * nb + b0 + i) * ngw;
                for (int g = 0; g < ngw; ++g) {
                    v[(size_t)(2 * i) * ngw + g] = cb[2 * g];
                    v[(size_t)(2 * i + 1) * ngw + g] = cb[2 * g + 1];
                }
            }
            memset(used, 0, (size_t)m);
            int deficient = 0;
            for (int s = 0; s < d; ++s) {
                int p = -1;
                double best = -1.0;
                for (int j = 0; j < m; ++j) {
                    if (used[j]) continue;
                    double nn = 0.0;
                    for (int g = 0; g < ngw; ++g) nn += v[(size_t)j * ngw + g] * v[(size_t)j * ngw + g];
                    if (nn > best) {
                        best = nn;
                        p = j;
                    }
                }
                double *q = r + ((size_t)k * nb + b0 + s) * ngw;
                if (p < 0 || !(best > 0.0)) { /* no vector left (or only NaN norms): not d real dimensions */
                    deficient = 1;
                    for (int g = 0; g < ngw; ++g) q[g] = 0.0;
                    continue;
                }
                used[p] = 1;
                const double inv = 1.0 / sqrt(best);
                for (int g = 0; g < ngw; ++g) q[g] = v[(size_t)p * ngw + g] * inv;
                for (int j = 0; j < m; ++j) {
                    if (used[j]) continue;
                    double dot = 0.0;
                    for (int g = 0; g < ngw; ++g) dot += q[g] * v[(size_t)j * ngw + g];
                    for (int g = 0; g < ngw; ++g) v[(size_t)j * ngw + g] -= dot * q[g];
                }
            }
            double rest = 0.0;
            for (int j = 0; j < m; ++j) {
                if (used[j]) continue;
                double nn = 0.0;
                for (int g = 0; g < ngw; ++g) nn += v[(size_t)j * ngw + g] * v[(size_t)j * ngw + g];
                if (nn > rest) rest = nn;
            }
            if (deficient || sqrt(rest) > 1e-6) ++bad;
            b0 = b1;
        }
    }
    free(v);
    free(used);
    return bad;
}
