/*
 * FP64 CPU oracle kernels for the PMMM far field (test infrastructure only).
 *
 * Nothing in the product path may link or call this file.  It is compiled
 * into oracle/liboracle.so and reached through oracle/exact.py and
 * oracle/pmmm.py from the tests, the package smoke check and the benchmark's
 * CPU-baseline leg.
 *
 * Contents
 *   ora_solid_S        singular solid harmonics S_l^m (App. A.1 definition,
 *                      evaluated with the App. A.5 scaled-Legendre recursion)
 *   ora_green_periodic periodic transfer-kernel mesh: the image sum of S_l^m
 *                      split with incomplete gamma functions (App. B,
 *                      eq. greenPBC), minus the image the near field covers
 *   ora_direct         open-boundary O(N^2) potential and gradient
 *   ora_ewald          Ewald reference (App. B, eq. refewald, with the charge
 *                      factor q_j in both sums and the self term -2a/sqrt(pi) q_i)
 *   ora_near           near-field direct sum over the (2c+1)^3 cells (Sec. 2.1)
 *
 * Conventions: Phi_i = sum_j q_j / |r_i - r_j|; the gradient returned is
 * grad Phi (not the force).  Real storage of a coefficient set follows
 * App. A.6: X[l(l+1)+m] = Re X_l^|m| for m >= 0 and Im X_l^|m| for m < 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_LMAX 32

static double fact_tab[2 * ORA_LMAX + 2];
static int fact_ready = 0;

static void init_fact(void) {
    if (fact_ready) return;
    fact_tab[0] = 1.0;
    for (int i = 1; i < 2 * ORA_LMAX + 2; ++i) fact_tab[i] = fact_tab[i - 1] * i;
    fact_ready = 1;
}

/* Scaled associated Legendre function Ptilde_l^m(r, z) (App. A.5) for
 * 0 <= m <= l <= lmax, written into P[l*(l+1)/2 + m]. */
static void scaled_legendre(int lmax, double r2, double z, double *P) {
    for (int m = 0; m <= lmax; ++m) {
        double dfact = 1.0; /* (2m-1)!! */
        for (int k = 1; k <= 2 * m - 1; k += 2) dfact *= k;
        double pmm = (m & 1) ? -dfact : dfact;
        P[m * (m + 1) / 2 + m] = pmm;
        if (m + 1 <= lmax) P[(m + 1) * (m + 2) / 2 + m] = (2 * m + 1) * z * pmm;
        for (int l = m + 2; l <= lmax; ++l) {
            double a = P[(l - 1) * l / 2 + m];
            double b = P[(l - 2) * (l - 1) / 2 + m];
            P[l * (l + 1) / 2 + m] = ((2 * l - 1) * z * a - (l + m - 1) * r2 * b) / (l - m);
        }
    }
}

/* S_l^m(x, y, z) for 0 <= m <= l <= lmax as complex numbers (re, im) at
 * index l*(l+1)/2 + m.  Uses S_l^{-m}(x,y,z) = (l-m)!/r^{2l+1} Q_l^m(-x,y,-z)
 * with Q_l^m = Ptilde_l^m (x + i y)^m, then S_l^m = (-1)^m conj(S_l^{-m}). */
void ora_solid_S(int lmax, double x, double y, double z, double *re, double *im) {
    init_fact();
    double P[(ORA_LMAX + 1) * (ORA_LMAX + 2) / 2];
    double r2 = x * x + y * y + z * z;
    double xm = -x, zm = -z; /* arguments of Q for S^{-m} */
    scaled_legendre(lmax, r2, zm, P);
    double rinv2 = 1.0 / r2, rinv = sqrt(rinv2);
    double pw_re = 1.0, pw_im = 0.0; /* (xm + i y)^m */
    for (int m = 0; m <= lmax; ++m) {
        double rpow = rinv; /* 1/r^{2l+1} starting at l = m */
        for (int k = 0; k < m; ++k) rpow *= rinv2;
        for (int l = m; l <= lmax; ++l) {
            int t = l * (l + 1) / 2 + m;
            double s = fact_tab[l - m] * rpow * P[t];
            /* S_l^{-m} = s * (xm + i y)^m */
            double sre = s * pw_re, sim = s * pw_im;
            /* S_l^m = (-1)^m conj(S_l^{-m}) */
            double sg = (m & 1) ? -1.0 : 1.0;
            re[t] = sg * sre;
            im[t] = -sg * sim;
            rpow *= rinv2;
        }
        double nre = pw_re * xm - pw_im * y;
        double nim = pw_re * y + pw_im * xm;
        pw_re = nre;
        pw_im = nim;
    }
}

/* Regularised upper incomplete gamma Q(l + 1/2, x) for l = 0..lmax by
 * Q(1/2, x) = erfc(sqrt x) and Q(a + 1, x) = Q(a, x) + x^a e^{-x} / Gamma(a + 1). */
static void inc_gamma_half(int lmax, double x, double *Qg) {
    double sx = sqrt(x);
    Qg[0] = erfc(sx);
    double gam = sqrt(M_PI); /* Gamma(1/2) */
    double xa = sx;          /* x^{1/2} */
    double ex = exp(-x);
    for (int l = 0; l < lmax; ++l) {
        double a = l + 0.5;
        gam *= a; /* Gamma(a + 1) */
        Qg[l + 1] = Qg[l] + xa * ex / gam;
        xa *= x;
    }
}

/* Regularised lower incomplete gamma P(l + 1/2, x) = 1 - Q(l + 1/2, x) for
 * l = 0..lmax.  Below x = a + 1 by its power series
 *     P(a, x) = x^a e^{-x} sum_{k >= 0} x^k / Gamma(a + k + 1),
 * which has no cancellation where P is small (near the origin and at high
 * order); above it as 1 - Q from inc_gamma_half. */
void ora_lower_gamma_half(int lmax, double x, double *P) {
    double Qg[2 * ORA_LMAX + 2];
    inc_gamma_half(lmax, x, Qg);
    double gam1 = 0.5 * sqrt(M_PI);  /* Gamma(a + 1) for a = 1/2 */
    double xa = sqrt(x);             /* x^a */
    const double ex = exp(-x);
    for (int l = 0; l <= lmax; ++l) {
        const double a = l + 0.5;
        if (x < a + 1.0) {
            double term = xa * ex / gam1, sum = 0.0;
            for (int k = 0; k < 400 && term > 1e-18 * sum; ++k) {
                sum += term;
                term *= x / (a + k + 1.0);
            }
            P[l] = sum;
        } else {
            P[l] = 1.0 - Qg[l];
        }
        xa *= x;
        gam1 *= a + 1.0;
    }
}

static inline int tri(int l, int m) { return l * (l + 1) / 2 + m; }

/* Periodic transfer-kernel mesh on an n^3 cell mesh of a cubic box of edge
 * `box`.  Output G[j][iz][iy][ix] in real storage for orders 0..lmax,
 * j < (lmax+1)^2, at the cell displacement delta = minimum image of
 * (ix, iy, iz), r = delta * h.
 *
 *   G(r) = sum_{|r + b n| <= nimg b} Q(l+1/2, a^2|r + b n|^2) S(r + b n)
 *        + sum_{0 < |n| <= nimg} (-i pi)^l / sqrt(pi) exp(-(pi k/a)^2)
 *              / Gamma(l+1/2) k^{2l-1} / V S(k_n) exp(2 pi i k_n . r)
 *
 * with k_n = n / b.  At delta = 0 the singular n = 0 real-space term is
 * left out (its smooth part stays in the reciprocal sum; the l = 0 limit is
 * removed later by the self correction).  For 0 < max|delta| <= cutoff the
 * one image covered by the near field, S(r), is subtracted: its real-space
 * term Q S(r) - S(r) is taken as -P(l+1/2, a^2 r^2) S(r), the same quantity
 * without the cancellation of two nearly equal large values. */
void ora_green_periodic(int n, double box, int lmax, int cutoff, double alpha, int nimg,
                        double *G) {
    init_fact();
    const int ntri = (lmax + 1) * (lmax + 2) / 2;
    const int Q = (lmax + 1) * (lmax + 1);
    const double h = box / n, V = box * box * box;
    const int64_t K = (int64_t)n * n * n;

    /* reciprocal vectors and their l-dependent prefactors, shared by all points */
    int nk = 0;
    for (int a = -nimg; a <= nimg; ++a)
        for (int b = -nimg; b <= nimg; ++b)
            for (int c = -nimg; c <= nimg; ++c)
                if ((a || b || c) && a * a + b * b + c * c <= nimg * nimg) ++nk;
    double *kv = (double *)malloc(sizeof(double) * 3 * nk);
    double *kre = (double *)malloc(sizeof(double) * nk * ntri);
    double *kim = (double *)malloc(sizeof(double) * nk * ntri);
    {
        int t = 0;
        for (int a = -nimg; a <= nimg; ++a)
            for (int b = -nimg; b <= nimg; ++b)
                for (int c = -nimg; c <= nimg; ++c) {
                    if (!(a || b || c) || a * a + b * b + c * c > nimg * nimg) continue;
                    double kx = a / box, ky = b / box, kz = c / box;
                    double kk = sqrt(kx * kx + ky * ky + kz * kz);
                    kv[3 * t] = kx;
                    kv[3 * t + 1] = ky;
                    kv[3 * t + 2] = kz;
                    double sre[ORA_LMAX * (ORA_LMAX + 1)], sim[ORA_LMAX * (ORA_LMAX + 1)];
                    ora_solid_S(lmax, kx, ky, kz, sre, sim);
                    double e = exp(-(M_PI * kk / alpha) * (M_PI * kk / alpha));
                    double gam = sqrt(M_PI); /* Gamma(l + 1/2) */
                    double kpow = 1.0 / kk;  /* k^{2l-1} */
                    /* (-i pi)^l as complex: cycle of (-i)^l */
                    double pil = 1.0;
                    for (int l = 0; l <= lmax; ++l) {
                        double coef = pil / sqrt(M_PI) * e / gam * kpow / V;
                        int ph = l & 3; /* (-i)^l: 1, -i, -1, i */
                        double cre = (ph == 0) ? coef : (ph == 2) ? -coef : 0.0;
                        double cim = (ph == 1) ? -coef : (ph == 3) ? coef : 0.0;
                        for (int m = 0; m <= l; ++m) {
                            int u = tri(l, m);
                            kre[(int64_t)t * ntri + u] = cre * sre[u] - cim * sim[u];
                            kim[(int64_t)t * ntri + u] = cre * sim[u] + cim * sre[u];
                        }
                        pil *= M_PI;
                        gam *= (l + 0.5);
                        kpow *= kk * kk;
                    }
                    ++t;
                }
    }

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t idx = 0; idx < K; ++idx) {
        int ix = (int)(idx % n), iy = (int)((idx / n) % n), iz = (int)(idx / ((int64_t)n * n));
        int dx = ix <= n / 2 ? ix : ix - n;
        int dy = iy <= n / 2 ? iy : iy - n;
        int dz = iz <= n / 2 ? iz : iz - n;
        double rx = dx * h, ry = dy * h, rz = dz * h;
        double accre[ORA_LMAX * (ORA_LMAX + 1)], accim[ORA_LMAX * (ORA_LMAX + 1)];
        double sre[ORA_LMAX * (ORA_LMAX + 1)], sim[ORA_LMAX * (ORA_LMAX + 1)];
        double Qg[ORA_LMAX + 2];
        for (int u = 0; u < ntri; ++u) accre[u] = accim[u] = 0.0;
        /* the near field covers the primary image of the near cells */
        int cheb = abs(dx);
        if (abs(dy) > cheb) cheb = abs(dy);
        if (abs(dz) > cheb) cheb = abs(dz);
        const int near = cheb > 0 && cheb <= cutoff;
        /* real-space images: every r + n b within nimg b of the origin (a
         * ball in distance, so the image sets of r and -r mirror each other
         * and do not depend on which image of a half-box offset is r) */
        const double rmax2 = (double)nimg * nimg * box * box;
        for (int a = -nimg - 1; a <= nimg + 1; ++a)
            for (int b = -nimg - 1; b <= nimg + 1; ++b)
                for (int c = -nimg - 1; c <= nimg + 1; ++c) {
                    if (dx == 0 && dy == 0 && dz == 0 && a == 0 && b == 0 && c == 0) continue;
                    double vx = rx + a * box, vy = ry + b * box, vz = rz + c * box;
                    double r2 = vx * vx + vy * vy + vz * vz;
                    if (r2 > rmax2) continue;
                    if (near && a == 0 && b == 0 && c == 0) {
                        /* Q S - S of the subtracted image = -P S */
                        ora_lower_gamma_half(lmax, alpha * alpha * r2, Qg);
                        for (int l = 0; l <= lmax; ++l) Qg[l] = -Qg[l];
                    } else {
                        inc_gamma_half(lmax, alpha * alpha * r2, Qg);
                    }
                    ora_solid_S(lmax, vx, vy, vz, sre, sim);
                    for (int l = 0; l <= lmax; ++l)
                        for (int m = 0; m <= l; ++m) {
                            int u = tri(l, m);
                            accre[u] += Qg[l] * sre[u];
                            accim[u] += Qg[l] * sim[u];
                        }
                }
        /* reciprocal images */
        for (int t = 0; t < nk; ++t) {
            double ph = 2.0 * M_PI * (kv[3 * t] * rx + kv[3 * t + 1] * ry + kv[3 * t + 2] * rz);
            double c = cos(ph), s = sin(ph);
            const double *kr = kre + (int64_t)t * ntri, *ki = kim + (int64_t)t * ntri;
            for (int u = 0; u < ntri; ++u) {
                accre[u] += kr[u] * c - ki[u] * s;
                accim[u] += kr[u] * s + ki[u] * c;
            }
        }
        for (int l = 0; l <= lmax; ++l) {
            for (int m = 0; m <= l; ++m) {
                int u = tri(l, m);
                G[(int64_t)(l * (l + 1) + m) * K + idx] = accre[u];
                if (m > 0) G[(int64_t)(l * (l + 1) - m) * K + idx] = accim[u];
            }
        }
    }
    (void)Q;
    free(kv);
    free(kre);
    free(kim);
}

/* Open boundary direct sum over all pairs j != i. */
void ora_direct(int64_t n, const double *pos, const double *q, double *phi, double *grad) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double p = 0, gx = 0, gy = 0, gz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            double ri = 1.0 / sqrt(r2);
            double qr = q[j] * ri;
            p += qr;
            double qr3 = qr * ri * ri;
            gx -= qr3 * dx;
            gy -= qr3 * dy;
            gz -= qr3 * dz;
        }
        phi[i] = p;
        grad[3 * i] = gx;
        grad[3 * i + 1] = gy;
        grad[3 * i + 2] = gz;
    }
}

/* The rows idx[0..m) of ora_direct: potential and gradient at the listed
 * particles from all other particles. */
void ora_direct_at(int64_t n, const double *pos, const double *q, int64_t m, const int64_t *idx,
                   double *phi, double *grad) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t i = idx[t];
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double p = 0, gx = 0, gy = 0, gz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            double ri = 1.0 / sqrt(r2);
            double qr = q[j] * ri;
            p += qr;
            double qr3 = qr * ri * ri;
            gx -= qr3 * dx;
            gy -= qr3 * dy;
            gz -= qr3 * dz;
        }
        phi[t] = p;
        grad[3 * t] = gx;
        grad[3 * t + 1] = gy;
        grad[3 * t + 2] = gz;
    }
}

/* Ewald reference for a cubic periodic box (tin-foil, no k = 0 term):
 *   Phi_i = sum'_{n,j} q_j erfc(a|r_ij + b n|)/|r_ij + b n|
 *         + 1/(pi V) sum_{k != 0} exp(-(pi k/a)^2)/k^2 Re sum_j q_j e^{2 pi i k . r_ij}
 *         - 2a/sqrt(pi) q_i - pi/(V a^2) sum_j q_j
 * Real space: images n in {-nr..nr}^3 with |r| < rcut; reciprocal space:
 * all integer vectors with 0 < |n| <= kmax (k = n / b). */
void ora_ewald(int64_t n, const double *pos, const double *q, double box, double alpha,
               int nr, double rcut, int kmax, double *phi, double *grad) {
    const double V = box * box * box;
    const double two_a_sqpi = 2.0 * alpha / sqrt(M_PI);
    double qtot = 0.0;
    for (int64_t j = 0; j < n; ++j) qtot += q[j];

    /* per-axis phase tables e^{2 pi i m x / b} for m = 0..kmax */
    const int nm = kmax + 1;
    double *cx = (double *)malloc(sizeof(double) * n * nm * 6);
    double *sx = cx + n * nm, *cy = sx + n * nm, *sy = cy + n * nm, *cz = sy + n * nm,
           *sz = cz + n * nm;
#pragma omp parallel for
    for (int64_t j = 0; j < n; ++j) {
        double ax = 2 * M_PI * pos[3 * j] / box, ay = 2 * M_PI * pos[3 * j + 1] / box,
               az = 2 * M_PI * pos[3 * j + 2] / box;
        for (int m = 0; m < nm; ++m) {
            cx[j * nm + m] = cos(m * ax);
            sx[j * nm + m] = sin(m * ax);
            cy[j * nm + m] = cos(m * ay);
            sy[j * nm + m] = sin(m * ay);
            cz[j * nm + m] = cos(m * az);
            sz[j * nm + m] = sin(m * az);
        }
    }
    /* half space of k: (a > 0) or (a == 0 && b > 0) or (a == 0 && b == 0 && c > 0) */
    int nk = 0;
    for (int a = 0; a <= kmax; ++a)
        for (int b = -kmax; b <= kmax; ++b)
            for (int c = -kmax; c <= kmax; ++c) {
                if (a * a + b * b + c * c > kmax * kmax) continue;
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                ++nk;
            }
    int *kl = (int *)malloc(sizeof(int) * 3 * nk);
    {
        int t = 0;
        for (int a = 0; a <= kmax; ++a)
            for (int b = -kmax; b <= kmax; ++b)
                for (int c = -kmax; c <= kmax; ++c) {
                    if (a * a + b * b + c * c > kmax * kmax) continue;
                    if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                    kl[3 * t] = a;
                    kl[3 * t + 1] = b;
                    kl[3 * t + 2] = c;
                    ++t;
                }
    }
    double *sre = (double *)calloc(nk, sizeof(double));
    double *sim = (double *)calloc(nk, sizeof(double));
    /* structure factors S(k) = sum_j q_j e^{2 pi i k . r_j} */
#pragma omp parallel for schedule(dynamic, 8)
    for (int t = 0; t < nk; ++t) {
        int a = kl[3 * t], b = kl[3 * t + 1], c = kl[3 * t + 2];
        int ab = abs(b), ac = abs(c);
        double sb = b < 0 ? -1.0 : 1.0, sc = c < 0 ? -1.0 : 1.0;
        double re = 0, im = 0;
        for (int64_t j = 0; j < n; ++j) {
            double c1 = cx[j * nm + a], s1 = sx[j * nm + a];
            double c2 = cy[j * nm + ab], s2 = sb * sy[j * nm + ab];
            double c3 = cz[j * nm + ac], s3 = sc * sz[j * nm + ac];
            double c12 = c1 * c2 - s1 * s2, s12 = s1 * c2 + c1 * s2;
            double cc = c12 * c3 - s12 * s3, ss = s12 * c3 + c12 * s3;
            re += q[j] * cc;
            im += q[j] * ss;
        }
        sre[t] = re;
        sim[t] = im;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double p = 0, gx = 0, gy = 0, gz = 0;
        /* real space; nr == 0 means minimum image (needs rcut <= b/2) */
        if (nr == 0) {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
                dx -= box * nearbyint(dx / box);
                dy -= box * nearbyint(dy / box);
                dz -= box * nearbyint(dz / box);
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 >= rcut * rcut) continue;
                double r = sqrt(r2);
                double ec = erfc(alpha * r) / r;
                p += q[j] * ec;
                double d = -(ec + two_a_sqpi * exp(-alpha * alpha * r2)) / r2;
                gx += q[j] * d * dx;
                gy += q[j] * d * dy;
                gz += q[j] * d * dz;
            }
        } else for (int64_t j = 0; j < n; ++j) {
            for (int a = -nr; a <= nr; ++a)
                for (int b = -nr; b <= nr; ++b)
                    for (int c = -nr; c <= nr; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double dx = xi - pos[3 * j] + a * box;
                        double dy = yi - pos[3 * j + 1] + b * box;
                        double dz = zi - pos[3 * j + 2] + c * box;
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 >= rcut * rcut) continue;
                        double r = sqrt(r2);
                        double ec = erfc(alpha * r) / r;
                        p += q[j] * ec;
                        double d = -(ec + two_a_sqpi * exp(-alpha * alpha * r2)) / r2;
                        gx += q[j] * d * dx;
                        gy += q[j] * d * dy;
                        gz += q[j] * d * dz;
                    }
        }
        /* reciprocal space: both k and -k, hence the factor 2 */
        for (int t = 0; t < nk; ++t) {
            int a = kl[3 * t], b = kl[3 * t + 1], c = kl[3 * t + 2];
            int ab = abs(b), ac = abs(c);
            double sb = b < 0 ? -1.0 : 1.0, sc = c < 0 ? -1.0 : 1.0;
            double c1 = cx[i * nm + a], s1 = sx[i * nm + a];
            double c2 = cy[i * nm + ab], s2 = sb * sy[i * nm + ab];
            double c3 = cz[i * nm + ac], s3 = sc * sz[i * nm + ac];
            double c12 = c1 * c2 - s1 * s2, s12 = s1 * c2 + c1 * s2;
            double cc = c12 * c3 - s12 * s3, ss = s12 * c3 + c12 * s3;
            double kx = a / box, ky = b / box, kz = c / box;
            double k2 = kx * kx + ky * ky + kz * kz;
            double w = 2.0 * exp(-(M_PI * M_PI * k2) / (alpha * alpha)) / (M_PI * V * k2);
            /* Re(e^{ik.ri} conj(S)) and its gradient */
            double re = cc * sre[t] + ss * sim[t];
            double im = ss * sre[t] - cc * sim[t];
            p += w * re;
            double g = -2.0 * M_PI * w * im;
            gx += g * kx;
            gy += g * ky;
            gz += g * kz;
        }
        p += -two_a_sqpi * q[i] - M_PI / (V * alpha * alpha) * qtot;
        phi[i] = p;
        grad[3 * i] = gx;
        grad[3 * i + 1] = gy;
        grad[3 * i + 2] = gz;
    }
    free(cx);
    free(kl);
    free(sre);
    free(sim);
}

/* Near field: for each particle i in cell I, the direct 1/r sum over the
 * particles j != i of the cells J with max_a |I_a - J_a| <= cutoff.
 * Periodic meshes wrap the cell offset and shift the partner by the
 * matching box vector (requires n >= 2 cutoff + 1).  `cell` holds each
 * particle's integer cell (ix, iy, iz); particles are given in any order. */
void ora_near(int64_t n, const double *pos, const double *q, const int *cell, int ncell,
              double box, int cutoff, int periodic, double *phi, double *grad) {
    const int64_t K = (int64_t)ncell * ncell * ncell;
    int64_t *cnt = (int64_t *)calloc(K + 1, sizeof(int64_t));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = ((int64_t)cell[3 * i + 2] * ncell + cell[3 * i + 1]) * ncell + cell[3 * i];
        cnt[c + 1]++;
    }
    for (int64_t c = 0; c < K; ++c) cnt[c + 1] += cnt[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (K > 0 ? K : 1));
    for (int64_t c = 0; c < K; ++c) fill[c] = cnt[c];
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = ((int64_t)cell[3 * i + 2] * ncell + cell[3 * i + 1]) * ncell + cell[3 * i];
        list[fill[c]++] = i;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double p = 0, gx = 0, gy = 0, gz = 0;
        int ci[3] = {cell[3 * i], cell[3 * i + 1], cell[3 * i + 2]};
        for (int oz = -cutoff; oz <= cutoff; ++oz)
            for (int oy = -cutoff; oy <= cutoff; ++oy)
                for (int ox = -cutoff; ox <= cutoff; ++ox) {
                    int cj[3] = {ci[0] + ox, ci[1] + oy, ci[2] + oz};
                    double sh[3] = {0, 0, 0};
                    int ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        if (cj[a] < 0 || cj[a] >= ncell) {
                            if (!periodic) {
                                ok = 0;
                                break;
                            }
                            if (cj[a] < 0) {
                                cj[a] += ncell;
                                sh[a] = -box;
                            } else {
                                cj[a] -= ncell;
                                sh[a] = box;
                            }
                        }
                    }
                    if (!ok) continue;
                    int64_t c = ((int64_t)cj[2] * ncell + cj[1]) * ncell + cj[0];
                    for (int64_t t = cnt[c]; t < cnt[c + 1]; ++t) {
                        int64_t j = list[t];
                        if (j == i) continue;
                        double dx = pos[3 * i] - (pos[3 * j] + sh[0]);
                        double dy = pos[3 * i + 1] - (pos[3 * j + 1] + sh[1]);
                        double dz = pos[3 * i + 2] - (pos[3 * j + 2] + sh[2]);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        double ri = 1.0 / sqrt(r2);
                        double qr = q[j] * ri;
                        p += qr;
                        double qr3 = qr * ri * ri;
                        gx -= qr3 * dx;
                        gy -= qr3 * dy;
                        gz -= qr3 * dz;
                    }
                }
        phi[i] = p;
        grad[3 * i] = gx;
        grad[3 * i + 1] = gy;
        grad[3 * i + 2] = gz;
    }
    free(cnt);
    free(list);
    free(fill);
}
