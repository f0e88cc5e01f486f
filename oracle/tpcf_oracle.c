/*
 * tpcf_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, double-precision CPU reference of the anisotropic 3PCF
 * estimator of arXiv:2408.03036, Sec. 4.2 (the Slepian-Eisenstein
 * pair-counting estimator), written from the paper's definitions:
 *
 *   a_lm(p, b)  = sum_{j in bin b of p} w_j conj(Y_lm(rhat_pj))      eq. (alm)
 *   local moments delta(x) a_l1m a*_l2m, with m = m' by the common line of
 *   sight along z                                               eq. (measured_mult)
 *   summed over all primaries ("average over positions")
 *   converted to the tripolar (TripoSH) multipoles with the Wigner 3j
 *   weights                                              eq. (slep2sugy), (TSHbasis)
 *
 * Only tests/, the package's smoke() and the benchmark's CPU-baseline leg may
 * load this file's library. It shares no code with the GPU library.
 *
 * Readings taken where the paper is silent:
 *  - bins are half-open [e_b, e_{b+1}); a pair is in bin b iff
 *    e_b^2 <= r^2 < e_{b+1}^2 with r^2 = dx*dx + dy*dy + dz*dz evaluated
 *    left to right in double (no fused multiply-add); r = 0 pairs are dropped;
 *  - periodic minimum image d -= L * rint(d / L) per axis (periodic boxes,
 *    Sec. 3 and Sec. 4);
 *  - the primary weight delta(x) of eq. (measured_mult) is w_p;
 *  - degenerate triangles (j == k) are removed, so the sums run over distinct
 *    triplets (flag subtract_self);
 *  - the normalisation is the analytic periodic-box count of random triplets,
 *    RRR(b1,b2) = N(N-1)(N-2) V_b1 V_b2 / L^6 (Sec. 4.1 states the analytic
 *    random counts for periodic boxes);
 *  - the output is the coefficient of the TripoSH basis of eq. (TSHbasis)
 *    (Schmidt semi-normalised y), so a Poisson catalogue gives c_000 = 1.
 *
 * The same file holds the anisotropic 2PCF of Sec. 4.1 (pair counts in
 * (r, mu), eq. (xi_natest), Legendre multipoles eq. (xi_meas_leg)); its
 * readings are listed with it below.
 *
 * Y_lm is orthonormal with the Condon-Shortley phase, evaluated from theta/phi
 * trigonometry and the textbook associated-Legendre recurrence in l.
 * The Wigner 3j symbols use Racah's single-sum formula.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- Y_lm */

/* P_l^m(x), 0 <= m <= l <= lmax, Condon-Shortley phase, stored at l*(lmax+1)+m.
 * P_m^m = (-1)^m (2m-1)!! (1-x^2)^{m/2};  P_{m+1}^m = x (2m+1) P_m^m;
 * (l-m) P_l^m = (2l-1) x P_{l-1}^m - (l+m-1) P_{l-2}^m. */
static void assoc_legendre(int lmax, double x, double* P)
{
    const int s1 = lmax + 1;
    double sth = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= -(2.0 * m - 1.0) * sth;
        P[m * s1 + m] = pmm;
        if (m == lmax) break;
        double p0 = pmm;
        double p1 = x * (2.0 * m + 1.0) * pmm;
        P[(m + 1) * s1 + m] = p1;
        for (int l = m + 2; l <= lmax; ++l) {
            double pl = ((2.0 * l - 1.0) * x * p1 - (l + m - 1.0) * p0) / (double)(l - m);
            P[l * s1 + m] = pl;
            p0 = p1;
            p1 = pl;
        }
    }
}

/* N_lm = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!) */
static double ylm_norm(int l, int m)
{
    double ratio = 1.0;
    for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
    return sqrt((2.0 * l + 1.0) / (4.0 * OR_PI) * ratio);
}

/* Y_lm(rhat) for 0 <= m <= l <= lmax at unit vector (x,y,z):
 * out[2*(l*(lmax+1)+m)] = Re, [+1] = Im. */
void oracle_ylm(int lmax, double x, double y, double z, double* out)
{
    const int s1 = lmax + 1;
    double* P = (double*)malloc(sizeof(double) * s1 * s1);
    double r = sqrt(x * x + y * y + z * z);
    double ct = z / r;
    double phi = atan2(y, x);
    assoc_legendre(lmax, ct, P);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m) {
            double v = ylm_norm(l, m) * P[l * s1 + m];
            out[2 * (l * s1 + m)] = v * cos(m * phi);
            out[2 * (l * s1 + m) + 1] = v * sin(m * phi);
        }
    free(P);
}

/* ---------------------------------------------------------------- 3j */

static long double lfact(int n)
{
    long double f = 1.0L;
    for (int k = 2; k <= n; ++k) f *= (long double)k;
    return f;
}

/* Racah's formula for (j1 j2 j3; m1 m2 m3), integer arguments. */
double oracle_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j1 < 0 || j2 < 0 || j3 < 0) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    if (j3 > j1 + j2 || j3 < abs(j1 - j2)) return 0.0;
    long double tri = lfact(j1 + j2 - j3) * lfact(j1 - j2 + j3) * lfact(-j1 + j2 + j3)
                      / lfact(j1 + j2 + j3 + 1);
    long double pre = sqrtl(tri * lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2)
                            * lfact(j2 - m2) * lfact(j3 + m3) * lfact(j3 - m3));
    int kmin = 0;
    if (j2 - j3 - m1 > kmin) kmin = j2 - j3 - m1;
    if (j1 - j3 + m2 > kmin) kmin = j1 - j3 + m2;
    int kmax = j1 + j2 - j3;
    if (j1 - m1 < kmax) kmax = j1 - m1;
    if (j2 + m2 < kmax) kmax = j2 + m2;
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        long double den = lfact(k) * lfact(j3 - j2 + k + m1) * lfact(j3 - j1 + k - m2)
                          * lfact(j1 + j2 - j3 - k) * lfact(j1 - k - m1) * lfact(j2 - k + m2);
        sum += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    int ph = j1 - j2 - m3;
    long double sgn = (((ph % 2) + 2) % 2) ? -1.0L : 1.0L;
    return (double)(sgn * pre * sum);
}

/* ---------------------------------------------------------------- estimator */

typedef struct {
    int64_t n;             /* number of points                                    */
    const double* pos;     /* (n,3) row-major                                     */
    const double* w;       /* (n) weights, NULL => all ones                       */
    double box;            /* periodic box side                                   */
    int nbins;             /* radial bins                                         */
    const double* edges;   /* nbins+1 increasing edges, edges[nbins] <= box/2     */
    int lmax;
    int subtract_self;     /* 1: distinct triplets only                           */
    int64_t prim_first;    /* primaries [prim_first, prim_first+prim_count)       */
    int64_t prim_count;    /* < 0 => all n                                        */
    int nthreads;          /* 0 => OpenMP default                                 */
} oracle_params;

static double wrap_coord(double x, double L)
{
    double y = fmod(x, L);
    if (y < 0.0) y += L;
    if (y >= L) y -= L;
    return y;
}

/* Index of the triple (m, l1, l2) in the (lmax+1)^3 NNN layout. */
#define NNN_IDX(m, l1, l2, s1) ((((m) * (s1) + (l1)) * (s1)) + (l2))

/*
 * Runs the estimator over the selected primaries.
 *  alm   : NULL or prim_count*nbins*(lmax+1)^2*2, layout [p][b][l][m] (re, im)
 *          holding a_lm(p,b) = sum_j w_j conj(Y_lm) for m <= l;
 *  nnn   : NULL or (lmax+1)^3 * nbins^2 * 2, layout [m][l1][l2][b1][b2] (re,im)
 *          holding NNN^m_{l1 l2}(b1,b2) = sum_p w_p [a_l1m(b1) conj(a_l2m(b2))
 *          - delta_{b1 b2} sum_j w_j^2 conj(Y_l1m) Y_l2m], m >= 0, l1,l2 >= m;
 *  npairs: NULL or the number of ordered in-shell pairs seen.
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_estimate(const oracle_params* prm, double* alm, double* nnn, int64_t* npairs)
{
    const int64_t n = prm->n;
    const double L = prm->box;
    const int nb = prm->nbins;
    const int lmax = prm->lmax;
    const int s1 = lmax + 1;
    if (n < 1 || !(L > 0.0) || nb < 1 || lmax < 0 || !prm->pos || !prm->edges) return -1;
    for (int b = 0; b < nb; ++b)
        if (!(prm->edges[b + 1] > prm->edges[b])) return -1;
    if (prm->edges[0] < 0.0 || prm->edges[nb] > 0.5 * L) return -1;
    int64_t p0 = prm->prim_first < 0 ? 0 : prm->prim_first;
    int64_t pc = prm->prim_count < 0 ? n - p0 : prm->prim_count;
    if (p0 + pc > n) return -1;

    double* x = (double*)malloc(sizeof(double) * 3 * n);
    for (int64_t i = 0; i < 3 * n; ++i) x[i] = wrap_coord(prm->pos[i], L);
    double* e2 = (double*)malloc(sizeof(double) * (nb + 1));
    for (int b = 0; b <= nb; ++b) e2[b] = prm->edges[b] * prm->edges[b];
    const double rmax = prm->edges[nb];

    /* Linked-list cell partition (Sec. 4.1): cells of side >= rmax, so every
     * in-shell neighbour lies in the 27 surrounding cells. Boxes with fewer
     * than 3 cells per side fall back to one cell holding everything. */
    int nc = (int)floor(L / rmax);
    if (nc < 3) nc = 1;
    const int64_t ncell = (int64_t)nc * nc * nc;
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * n);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int cx = (int)(x[3 * i] / L * nc), cy = (int)(x[3 * i + 1] / L * nc),
            cz = (int)(x[3 * i + 2] / L * nc);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        if (cz >= nc) cz = nc - 1;
        int64_t c = ((int64_t)cx * nc + cy) * nc + cz;
        next[i] = head[c];
        head[c] = i;
    }

    double* Ntab = (double*)malloc(sizeof(double) * s1 * s1);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m) Ntab[l * s1 + m] = ylm_norm(l, m);

    const size_t nnn_sz = (size_t)s1 * s1 * s1 * nb * nb * 2;
    int nthr = 1;
#ifdef _OPENMP
    nthr = prm->nthreads > 0 ? prm->nthreads : omp_get_max_threads();
#endif
    double* nnn_thr = NULL;
    if (nnn) {
        nnn_thr = (double*)calloc((size_t)nthr * nnn_sz, sizeof(double));
    }
    int64_t* np_thr = (int64_t*)calloc((size_t)nthr, sizeof(int64_t));

#ifdef _OPENMP
#pragma omp parallel num_threads(nthr)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* P = (double*)malloc(sizeof(double) * s1 * s1);
        double* are = (double*)malloc(sizeof(double) * nb * s1 * s1);
        double* aim = (double*)malloc(sizeof(double) * nb * s1 * s1);
        /* self[b][m][l1][l2] = sum_j w_j^2 conj(Y_l1m) Y_l2m  (real) */
        double* self = (double*)malloc(sizeof(double) * nb * s1 * s1 * s1);
        double* yre = (double*)malloc(sizeof(double) * s1 * s1);
        double* yim = (double*)malloc(sizeof(double) * s1 * s1);
        double* mynnn = nnn_thr ? nnn_thr + (size_t)tid * nnn_sz : NULL;
        int64_t mypairs = 0;

#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t ip = 0; ip < pc; ++ip) {
            const int64_t p = p0 + ip;
            memset(are, 0, sizeof(double) * nb * s1 * s1);
            memset(aim, 0, sizeof(double) * nb * s1 * s1);
            memset(self, 0, sizeof(double) * nb * s1 * s1 * s1);
            const double xp = x[3 * p], yp = x[3 * p + 1], zp = x[3 * p + 2];
            int cx = (int)(xp / L * nc), cy = (int)(yp / L * nc), cz = (int)(zp / L * nc);
            if (cx >= nc) cx = nc - 1;
            if (cy >= nc) cy = nc - 1;
            if (cz >= nc) cz = nc - 1;
            const int span = nc == 1 ? 0 : 1;
            for (int ox = -span; ox <= span; ++ox)
                for (int oy = -span; oy <= span; ++oy)
                    for (int oz = -span; oz <= span; ++oz) {
                        int qx = (cx + ox + nc) % nc, qy = (cy + oy + nc) % nc,
                            qz = (cz + oz + nc) % nc;
                        int64_t c = ((int64_t)qx * nc + qy) * nc + qz;
                        for (int64_t j = head[c]; j >= 0; j = next[j]) {
                            if (j == p) continue;
                            double dx = x[3 * j] - xp, dy = x[3 * j + 1] - yp,
                                   dz = x[3 * j + 2] - zp;
                            dx -= L * rint(dx / L);
                            dy -= L * rint(dy / L);
                            dz -= L * rint(dz / L);
                            double r2 = dx * dx;
                            r2 += dy * dy;
                            r2 += dz * dz;
                            if (r2 == 0.0) continue;
                            if (r2 < e2[0] || r2 >= e2[nb]) continue;
                            int b = 0;
                            while (!(r2 >= e2[b] && r2 < e2[b + 1])) ++b;
                            ++mypairs;
                            const double wj = prm->w ? prm->w[j] : 1.0;
                            const double r = sqrt(r2);
                            const double ct = dz / r;
                            const double phi = atan2(dy, dx);
                            assoc_legendre(lmax, ct, P);
                            for (int l = 0; l <= lmax; ++l)
                                for (int m = 0; m <= l; ++m) {
                                    double v = Ntab[l * s1 + m] * P[l * s1 + m];
                                    yre[l * s1 + m] = v * cos(m * phi);
                                    yim[l * s1 + m] = v * sin(m * phi);
                                }
                            double* ar = are + (size_t)b * s1 * s1;
                            double* ai = aim + (size_t)b * s1 * s1;
                            for (int l = 0; l <= lmax; ++l)
                                for (int m = 0; m <= l; ++m) {
                                    /* w_j conj(Y_lm) */
                                    ar[l * s1 + m] += wj * yre[l * s1 + m];
                                    ai[l * s1 + m] -= wj * yim[l * s1 + m];
                                }
                            double* sf = self + (size_t)b * s1 * s1 * s1;
                            const double w2 = wj * wj;
                            for (int m = 0; m <= lmax; ++m)
                                for (int l1 = m; l1 <= lmax; ++l1)
                                    for (int l2 = m; l2 <= lmax; ++l2) {
                                        /* Re(conj(Y1) Y2); conj(Y1) Y2 is real for equal m */
                                        double v = yre[l1 * s1 + m] * yre[l2 * s1 + m]
                                                   + yim[l1 * s1 + m] * yim[l2 * s1 + m];
                                        sf[NNN_IDX(m, l1, l2, s1)] += w2 * v;
                                    }
                        }
                    }
            if (alm) {
                double* out = alm + (size_t)ip * nb * s1 * s1 * 2;
                for (int b = 0; b < nb; ++b)
                    for (int k = 0; k < s1 * s1; ++k) {
                        out[2 * (b * s1 * s1 + k)] = are[b * s1 * s1 + k];
                        out[2 * (b * s1 * s1 + k) + 1] = aim[b * s1 * s1 + k];
                    }
            }
            if (mynnn) {
                const double wp = prm->w ? prm->w[p] : 1.0;
                for (int m = 0; m <= lmax; ++m)
                    for (int l1 = m; l1 <= lmax; ++l1)
                        for (int l2 = m; l2 <= lmax; ++l2) {
                            double* o = mynnn + (size_t)NNN_IDX(m, l1, l2, s1) * nb * nb * 2;
                            for (int b1 = 0; b1 < nb; ++b1) {
                                const double a1r = are[b1 * s1 * s1 + l1 * s1 + m];
                                const double a1i = aim[b1 * s1 * s1 + l1 * s1 + m];
                                for (int b2 = 0; b2 < nb; ++b2) {
                                    const double a2r = are[b2 * s1 * s1 + l2 * s1 + m];
                                    const double a2i = aim[b2 * s1 * s1 + l2 * s1 + m];
                                    /* a1 * conj(a2) */
                                    double re = a1r * a2r + a1i * a2i;
                                    double im = a1i * a2r - a1r * a2i;
                                    if (b1 == b2 && prm->subtract_self)
                                        re -= self[(size_t)b1 * s1 * s1 * s1 + NNN_IDX(m, l1, l2, s1)];
                                    o[2 * (b1 * nb + b2)] += wp * re;
                                    o[2 * (b1 * nb + b2) + 1] += wp * im;
                                }
                            }
                        }
            }
        }
        np_thr[tid] = mypairs;
        free(P);
        free(are);
        free(aim);
        free(self);
        free(yre);
        free(yim);
    }

    if (nnn) {
        memset(nnn, 0, sizeof(double) * nnn_sz);
        for (int t = 0; t < nthr; ++t)
            for (size_t k = 0; k < nnn_sz; ++k) nnn[k] += nnn_thr[(size_t)t * nnn_sz + k];
        free(nnn_thr);
    }
    if (npairs) {
        int64_t s = 0;
        for (int t = 0; t < nthr; ++t) s += np_thr[t];
        *npairs = s;
    }
    free(np_thr);
    free(Ntab);
    free(head);
    free(next);
    free(e2);
    free(x);
    return 0;
}

/*
 * TripoSH multipoles from the NNN^m moments (eq. (slep2sugy), (TSHbasis)):
 *   c_{l1 l2 L}(b1,b2) = 4 pi sqrt((2l1+1)(2l2+1)) (2L+1) H_{l1 l2 L}
 *        * sum_{m=-min(l1,l2)}^{min} (l1 l2 L; m -m 0) (-1)^m NNN^m(b1,b2) / RRR(b1,b2)
 * with NNN^{-m} = conj(NNN^m) (because Y_{l,-m} = (-1)^m conj(Y_lm)), and
 *   RRR(b1,b2) = n_data (n_data-1)(n_data-2) V_b1 V_b2 / L^6.
 * literal != 0 returns instead eq. (slep2sugy) as printed, applied to the
 * orthonormal-Y coefficients zeta^m = (4 pi)^2 NNN^m / RRR.
 * out_re/out_im: n_mult * nbins * nbins. Returns 0 or -1.
 */
int oracle_multipoles(const double* nnn, int64_t n_data, double box, int nbins,
                      const double* edges, int lmax, int n_mult, const int* l1l2L,
                      int literal, double* out_re, double* out_im)
{
    const int s1 = lmax + 1;
    const int nb = nbins;
    if (n_data < 3) return -1;
    double* V = (double*)malloc(sizeof(double) * nb);
    for (int b = 0; b < nb; ++b)
        V[b] = 4.0 * OR_PI / 3.0 * (edges[b + 1] * edges[b + 1] * edges[b + 1]
                                    - edges[b] * edges[b] * edges[b]);
    const double nd = (double)n_data;
    const double L3 = box * box * box;
    for (int t = 0; t < n_mult; ++t) {
        const int l1 = l1l2L[3 * t], l2 = l1l2L[3 * t + 1], LL = l1l2L[3 * t + 2];
        if (l1 < 0 || l2 < 0 || l1 > lmax || l2 > lmax || LL < abs(l1 - l2) || LL > l1 + l2
            || ((l1 + l2 + LL) & 1)) {
            free(V);
            return -1;
        }
        const double H = oracle_wigner3j(l1, l2, LL, 0, 0, 0);
        const double pref = literal
            ? (2.0 * LL + 1.0) * H * 16.0 * OR_PI * OR_PI
            : 4.0 * OR_PI * sqrt((2.0 * l1 + 1.0) * (2.0 * l2 + 1.0)) * (2.0 * LL + 1.0) * H;
        const int mm = l1 < l2 ? l1 : l2;
        for (int b1 = 0; b1 < nb; ++b1)
            for (int b2 = 0; b2 < nb; ++b2) {
                double sre = 0.0, sim = 0.0;
                for (int m = -mm; m <= mm; ++m) {
                    const int am = abs(m);
                    const double* v = nnn + ((size_t)NNN_IDX(am, l1, l2, s1) * nb * nb
                                             + (size_t)b1 * nb + b2) * 2;
                    const double re = v[0];
                    const double im = m < 0 ? -v[1] : v[1];
                    const double cg = oracle_wigner3j(l1, l2, LL, m, -m, 0) * ((am & 1) ? -1.0 : 1.0);
                    sre += cg * re;
                    sim += cg * im;
                }
                const double rrr = nd * (nd - 1.0) * (nd - 2.0) * V[b1] * V[b2] / (L3 * L3);
                out_re[((size_t)t * nb + b1) * nb + b2] = pref * sre / rrr;
                if (out_im) out_im[((size_t)t * nb + b1) * nb + b2] = pref * sim / rrr;
            }
    }
    free(V);
    return 0;
}

/* ================================================================ 2PCF
 *
 * Anisotropic two-point function of Sec. 4.1: pair counts DD(r, mu) in bins
 * of separation r and of mu = rhat . z (the common line of sight along z),
 * the natural estimator xi(r, mu) = DD / RR - 1 of eq. (xi_natest) with the
 * analytic random-pair counts of a periodic box, and its Legendre multipoles
 * of eq. (xi_meas_leg).
 *
 * Readings taken where the paper is silent:
 *  - pairs are ordered (p, j) with j != p; the radial bin is that of the
 *    3PCF above (half-open, from r^2 = dx*dx + dy*dy + dz*dz evaluated left
 *    to right, minimum image, r = 0 dropped);
 *  - mu covers [-1, 1] in nmu equal bins; with r = sqrt(r^2) and
 *    mu = dz / r the bin is k = floor((mu + 1) * (nmu / 2)), every operation
 *    rounded in double, and k is clamped to [0, nmu - 1] (so mu = 1 falls in
 *    the last bin);
 *  - RR(b, k) = N (N - 1) V_b / (nmu L^3): N (N - 1) ordered pairs of
 *    uniform points, the fraction V_b / L^3 of them in shell b (exact for
 *    e_nb <= L/2) spread evenly over mu;
 *  - xi(r, mu) is constant inside a mu bin, so the integral of eq.
 *    (xi_meas_leg) becomes sum_k xi(r_b, mu_k) times the exact integral of
 *    P_l over the bin.
 */

/* P_l(x) for l = 0..lmax by Bonnet's recurrence (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}. */
static void legendre_all(int lmax, double x, double* P)
{
    P[0] = 1.0;
    if (lmax >= 1) P[1] = x;
    for (int l = 1; l < lmax; ++l)
        P[l + 1] = ((2.0 * l + 1.0) * x * P[l] - (double)l * P[l - 1]) / (double)(l + 1);
}

/* Integral of P_l over [a, b]: b - a for l = 0, otherwise
 * [P_{l+1} - P_{l-1}] / (2l + 1) between a and b (from
 * (2l+1) P_l = d/dx (P_{l+1} - P_{l-1})). */
double oracle_legendre_bin_integral(int l, double a, double b)
{
    if (l < 0) return 0.0;
    if (l == 0) return b - a;
    double Pa[64], Pb[64];
    if (l + 1 >= 64) return 0.0;
    legendre_all(l + 1, a, Pa);
    legendre_all(l + 1, b, Pb);
    return ((Pb[l + 1] - Pb[l - 1]) - (Pa[l + 1] - Pa[l - 1])) / (2.0 * l + 1.0);
}

/*
 * DD(r, mu) of the points (pos, n) in a periodic box: counts[b * nmu + k]
 * (int64) of ordered pairs in radial bin b and mu bin k.
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_xi_counts(int64_t n, const double* pos, double box, int nbins, const double* edges,
                     int nmu, int nthreads, int64_t* counts)
{
    const double L = box;
    const int nb = nbins;
    if (n < 1 || !(L > 0.0) || nb < 1 || nmu < 1 || !pos || !edges || !counts) return -1;
    for (int b = 0; b < nb; ++b)
        if (!(edges[b + 1] > edges[b])) return -1;
    if (edges[0] < 0.0 || edges[nb] > 0.5 * L) return -1;

    double* x = (double*)malloc(sizeof(double) * 3 * n);
    for (int64_t i = 0; i < 3 * n; ++i) x[i] = wrap_coord(pos[i], L);
    double* e2 = (double*)malloc(sizeof(double) * (nb + 1));
    for (int b = 0; b <= nb; ++b) e2[b] = edges[b] * edges[b];
    const double half = (double)nmu / 2.0;

    /* Linked-list cell partition with cells of side >= r_max (27 neighbour
     * cells), or one cell when the box holds fewer than 3 per side. */
    int nc = (int)floor(L / edges[nb]);
    if (nc < 3) nc = 1;
    const int64_t ncell = (int64_t)nc * nc * nc;
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * n);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int cx = (int)(x[3 * i] / L * nc), cy = (int)(x[3 * i + 1] / L * nc),
            cz = (int)(x[3 * i + 2] / L * nc);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        if (cz >= nc) cz = nc - 1;
        int64_t c = ((int64_t)cx * nc + cy) * nc + cz;
        next[i] = head[c];
        head[c] = i;
    }

    const size_t nh = (size_t)nb * nmu;
    int nthr = 1;
#ifdef _OPENMP
    nthr = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    int64_t* hist = (int64_t*)calloc((size_t)nthr * nh, sizeof(int64_t));

#ifdef _OPENMP
#pragma omp parallel num_threads(nthr)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t* my = hist + (size_t)tid * nh;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
        for (int64_t p = 0; p < n; ++p) {
            const double xp = x[3 * p], yp = x[3 * p + 1], zp = x[3 * p + 2];
            int cx = (int)(xp / L * nc), cy = (int)(yp / L * nc), cz = (int)(zp / L * nc);
            if (cx >= nc) cx = nc - 1;
            if (cy >= nc) cy = nc - 1;
            if (cz >= nc) cz = nc - 1;
            const int span = nc == 1 ? 0 : 1;
            for (int ox = -span; ox <= span; ++ox)
                for (int oy = -span; oy <= span; ++oy)
                    for (int oz = -span; oz <= span; ++oz) {
                        int qx = (cx + ox + nc) % nc, qy = (cy + oy + nc) % nc,
                            qz = (cz + oz + nc) % nc;
                        int64_t c = ((int64_t)qx * nc + qy) * nc + qz;
                        for (int64_t j = head[c]; j >= 0; j = next[j]) {
                            if (j == p) continue;
                            double dx = x[3 * j] - xp, dy = x[3 * j + 1] - yp,
                                   dz = x[3 * j + 2] - zp;
                            dx -= L * rint(dx / L);
                            dy -= L * rint(dy / L);
                            dz -= L * rint(dz / L);
                            double r2 = dx * dx;
                            r2 += dy * dy;
                            r2 += dz * dz;
                            if (r2 == 0.0) continue;
                            if (r2 < e2[0] || r2 >= e2[nb]) continue;
                            int b = 0;
                            while (!(r2 >= e2[b] && r2 < e2[b + 1])) ++b;
                            const double r = sqrt(r2);
                            const double mu = dz / r;
                            const double t = (mu + 1.0) * half;
                            int k = (int)floor(t);
                            if (k < 0) k = 0;
                            if (k > nmu - 1) k = nmu - 1;
                            my[(size_t)b * nmu + k] += 1;
                        }
                    }
        }
    }
    for (size_t i = 0; i < nh; ++i) {
        int64_t s = 0;
        for (int t = 0; t < nthr; ++t) s += hist[(size_t)t * nh + i];
        counts[i] = s;
    }
    free(hist);
    free(head);
    free(next);
    free(e2);
    free(x);
    return 0;
}

/*
 * Legendre multipoles of the natural estimator (eq. (xi_natest), (xi_meas_leg)):
 *   xi(r_b, mu_k) = DD(b, k) / RR(b, k) - 1,  RR(b, k) = N (N-1) V_b / (nmu L^3),
 *   xi_l(r_b) = (2l + 1) / 2 * sum_k xi(r_b, mu_k) * integral of P_l over bin k,
 * with the mu bin edges mu_k = -1 + 2k / nmu.
 * out: n_ell * nbins, [i][b] for l = ells[i]. Returns 0 or -1.
 */
int oracle_xi_multipoles(const int64_t* counts, int64_t n_data, double box, int nbins,
                         const double* edges, int nmu, int n_ell, const int* ells, double* out)
{
    if (n_data < 2 || !(box > 0.0) || nbins < 1 || nmu < 1 || n_ell < 0) return -1;
    const double nd = (double)n_data;
    const double L3 = box * box * box;
    for (int i = 0; i < n_ell; ++i) {
        const int l = ells[i];
        if (l < 0 || l > 60) return -1;
        for (int b = 0; b < nbins; ++b) {
            const double V = 4.0 * OR_PI / 3.0 *
                             (edges[b + 1] * edges[b + 1] * edges[b + 1] - edges[b] * edges[b] * edges[b]);
            const double rr = nd * (nd - 1.0) * V / ((double)nmu * L3);
            double s = 0.0;
            for (int k = 0; k < nmu; ++k) {
                const double lo = -1.0 + 2.0 * (double)k / (double)nmu;
                const double hi = -1.0 + 2.0 * (double)(k + 1) / (double)nmu;
                const double xi = (double)counts[(size_t)b * nmu + k] / rr - 1.0;
                s += xi * oracle_legendre_bin_integral(l, lo, hi);
            }
            out[(size_t)i * nbins + b] = (2.0 * l + 1.0) / 2.0 * s;
        }
    }
    return 0;
}
