/*
 * Plain FP64 CPU oracle for the AO -> MO value / gradient / Laplacian path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, calls or includes
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code with the GPU path.
 *
 * It is deliberately slow and literal: every primitive of every shell is
 * visited for every point, sums run in input order, and no blocking, fusion
 * or reordering is done beyond what the definitions state.
 *
 * Definitions followed (QMCkl paper, arXiv 2512.16677):
 *   - AO as normalisation x radial x angular part: Section 3.1, first equation
 *     (chi_n = M_n R_theta(n) P_eta(n)).
 *   - Radial part as a contraction of Gaussian primitives (p = 2, n_s = 0):
 *     Section 3.1, second equation.
 *   - Exponent cutoff with the precision parameter B (default 53): Section
 *     3.1, third equation; a primitive whose argument fails the test
 *     contributes zero to the value and to every derivative.
 *   - Angular part P = (x-X_A)^a (y-Y_A)^b (z-Z_A)^c: Section 3.1, fourth
 *     equation.
 *   - MO value, gradient, Laplacian as C-weighted sums of the AO ones:
 *     Section 3.2, equations for phi_n, grad phi_n, Laplacian phi_n.
 *   - Derivatives up to third order for forces / parameter derivatives:
 *     Section 3.6 and Section 3.5 (last paragraph) motivate the adjoint.
 *
 * Readings where the paper is silent (each one is listed in the design
 * notes): natural log in the cutoff, strict "<" (equality gives zero); the
 * normalisation f, N_s, M_n makes every Cartesian AO unit-norm; Cartesian
 * components of a shell ordered lexicographically with the x power
 * descending (d: xx xy xz yy yz zz); output components ordered
 * (value, d/dx, d/dy, d/dz, Laplacian).  B <= 0 disables the cutoff.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846

/* (n)!! for odd n >= -1, with (-1)!! = 1. */
static double odd_double_factorial(int n) {
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= (double)k;
    return r;
}

static int n_cart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents (a,b,c) of component `i` of a shell of angular
 * momentum l: a descending from l, then b descending, c = l - a - b. */
static void cart_powers(int l, int i, int* a, int* b, int* c) {
    int idx = 0;
    for (int aa = l; aa >= 0; --aa)
        for (int bb = l - aa; bb >= 0; --bb) {
            if (idx == i) { *a = aa; *b = bb; *c = l - aa - bb; return; }
            ++idx;
        }
}

/* x^n for n >= 0, zero for n < 0 (a derivative that removes the power). */
static double ipow(double x, int n) {
    if (n < 0) return 0.0;
    double r = 1.0;
    for (int k = 0; k < n; ++k) r *= x;
    return r;
}

int64_t oracle_ao_num(int64_t shell_num, const int32_t* shell_ang_mom) {
    int64_t n = 0;
    for (int64_t s = 0; s < shell_num; ++s) n += n_cart(shell_ang_mom[s]);
    return n;
}

/*
 * Normalisation factors (Section 3.1, the factors f_ks, N_s, M_n).
 *   f_k = (2 g/pi)^(3/4) (4 g)^(l/2) / sqrt((2l-1)!!)   normalises the
 *         axis-aligned primitive x^l exp(-g r^2);
 *   N_s = [ sum_kl a_k a_l f_k f_l (pi/(g_k+g_l))^(3/2) (2l-1)!!
 *                                    / (2 (g_k+g_l))^l ]^(-1/2)
 *         normalises the contracted axis-aligned function;
 *   M_(a,b,c) = sqrt((2l-1)!! / ((2a-1)!! (2b-1)!! (2c-1)!!))
 *         carries the axis normalisation to every Cartesian component.
 */
void oracle_normalisation(int64_t shell_num, const int32_t* shell_ang_mom,
                          const int64_t* shell_prim_offset, const double* exponent,
                          const double* coefficient, double* prim_factor,
                          double* shell_factor, double* ao_factor) {
    int64_t ao = 0;
    for (int64_t s = 0; s < shell_num; ++s) {
        int l = shell_ang_mom[s];
        double dfl = odd_double_factorial(2 * l - 1);
        for (int64_t k = shell_prim_offset[s]; k < shell_prim_offset[s + 1]; ++k) {
            double g = exponent[k];
            prim_factor[k] = pow(2.0 * g / ORACLE_PI, 0.75) * pow(4.0 * g, 0.5 * l) / sqrt(dfl);
        }
        double ovl = 0.0;
        for (int64_t k = shell_prim_offset[s]; k < shell_prim_offset[s + 1]; ++k)
            for (int64_t q = shell_prim_offset[s]; q < shell_prim_offset[s + 1]; ++q) {
                double al = exponent[k] + exponent[q];
                ovl += coefficient[k] * coefficient[q] * prim_factor[k] * prim_factor[q] *
                       pow(ORACLE_PI / al, 1.5) * dfl / pow(2.0 * al, (double)l);
            }
        shell_factor[s] = 1.0 / sqrt(ovl);
        for (int i = 0; i < n_cart(l); ++i) {
            int a, b, c;
            cart_powers(l, i, &a, &b, &c);
            ao_factor[ao++] = sqrt(dfl / (odd_double_factorial(2 * a - 1) *
                                          odd_double_factorial(2 * b - 1) *
                                          odd_double_factorial(2 * c - 1)));
        }
    }
}

/* Number of derivative quantities returned per AO by oracle_ao_derivs. */
#define ORACLE_NQ 14
/* Quantity order: 0 value; 1..3 d/dx, d/dy, d/dz; 4 Laplacian;
 * 5..10 Hessian xx xy xz yy yz zz; 11..13 d/dx, d/dy, d/dz of the Laplacian. */

/*
 * Derivatives of the angular monomial P = x^a y^b z^c at displacement d.
 * dP[i] = dP/dd_i, hP[i][j], lP = Laplacian, glP[i] = d/dd_i Laplacian.
 */
static void monomial_derivs(int a, int b, int c, const double d[3], double* P, double dP[3],
                            double hP[3][3], double* lP, double glP[3]) {
    int e[3] = {a, b, c};
    /* f(n, m): m-th derivative coefficient of t^n is n (n-1) .. (n-m+1) t^(n-m). */
    double v[3][4]; /* v[axis][m] = m-th derivative of d_axis^e_axis */
    for (int ax = 0; ax < 3; ++ax)
        for (int m = 0; m < 4; ++m) {
            double coef = 1.0;
            for (int q = 0; q < m; ++q) coef *= (double)(e[ax] - q);
            v[ax][m] = coef * ipow(d[ax], e[ax] - m);
        }
    *P = v[0][0] * v[1][0] * v[2][0];
    dP[0] = v[0][1] * v[1][0] * v[2][0];
    dP[1] = v[0][0] * v[1][1] * v[2][0];
    dP[2] = v[0][0] * v[1][0] * v[2][1];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int m[3] = {0, 0, 0};
            m[i] += 1;
            m[j] += 1;
            hP[i][j] = v[0][m[0]] * v[1][m[1]] * v[2][m[2]];
        }
    *lP = hP[0][0] + hP[1][1] + hP[2][2];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) {
            int m[3] = {0, 0, 0};
            m[i] += 1;
            m[j] += 2;
            s += v[0][m[0]] * v[1][m[1]] * v[2][m[2]];
        }
        glP[i] = s;
    }
}

/*
 * AO values and derivatives at `point_num` points.
 *   out[p][q][k], q in 0..ORACLE_NQ-1 (see above) if nq == ORACLE_NQ,
 *   or only q in 0..4 (value, gradient, Laplacian) if nq == 5.
 * Each AO is chi = M P(d) R(u), d = r - R_A, u = |d|^2,
 * R(u) = N_s sum_k a_k f_k exp(-g_k u) over primitives with g_k u < T,
 * T = (B-1) ln 2.  With g0..g3 the u-derivatives of R of order 0..3:
 *   d_i chi      = M (d_iP g0 + 2 d_i P g1)
 *   d_i d_j chi  = M (d_i d_j P g0 + 2 (d_j d_iP + d_i d_jP) g1
 *                     + 2 delta_ij P g1 + 4 d_i d_j P g2)
 *   lap chi      = M (lap P g0 + (4l+6) P g1 + 4 u P g2)      (x.grad P = l P)
 *   d_i lap chi  = M (d_i lapP g0 + (2 d_i lapP + (4l+6) d_iP) g1
 *                     + ((8l+20) d_i P + 4 u d_iP) g2 + 8 u d_i P g3).
 */
int oracle_ao_derivs(int64_t nucl_num, const double* nucl_coord, int64_t shell_num,
                     const int64_t* shell_nucleus, const int32_t* shell_ang_mom,
                     const int64_t* shell_prim_offset, const double* exponent,
                     const double* coefficient, int64_t point_num, const double* point,
                     double B, int nq, double* out) {
    if (nq != 5 && nq != ORACLE_NQ) return 1;
    int64_t prim_num = shell_prim_offset[shell_num];
    int64_t ao_num = oracle_ao_num(shell_num, shell_ang_mom);
    double* f = (double*)malloc(sizeof(double) * (size_t)(prim_num > 0 ? prim_num : 1));
    double* ns = (double*)malloc(sizeof(double) * (size_t)(shell_num > 0 ? shell_num : 1));
    double* m = (double*)malloc(sizeof(double) * (size_t)(ao_num > 0 ? ao_num : 1));
    if (!f || !ns || !m) { free(f); free(ns); free(m); return 2; }
    for (int64_t s = 0; s < shell_num; ++s)
        if (shell_nucleus[s] < 0 || shell_nucleus[s] >= nucl_num) { free(f); free(ns); free(m); return 3; }
    oracle_normalisation(shell_num, shell_ang_mom, shell_prim_offset, exponent, coefficient, f, ns, m);
    double T = (B > 0.0) ? (B - 1.0) * log(2.0) : INFINITY;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < point_num; ++p) {
        double* o = out + (size_t)p * (size_t)nq * (size_t)ao_num;
        int64_t ao = 0;
        for (int64_t s = 0; s < shell_num; ++s) {
            int l = shell_ang_mom[s];
            const double* R = nucl_coord + 3 * shell_nucleus[s];
            double d[3] = {point[3 * p + 0] - R[0], point[3 * p + 1] - R[1], point[3 * p + 2] - R[2]};
            double u = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
            for (int64_t k = shell_prim_offset[s]; k < shell_prim_offset[s + 1]; ++k) {
                double x = exponent[k] * u;
                if (!(x < T)) continue; /* cutoff: primitive and derivatives are zero */
                double e = coefficient[k] * f[k] * ns[s] * exp(-x);
                double g = exponent[k];
                g0 += e;
                g1 += -g * e;
                g2 += g * g * e;
                g3 += -g * g * g * e;
            }
            for (int i = 0; i < n_cart(l); ++i, ++ao) {
                int a, b, c;
                cart_powers(l, i, &a, &b, &c);
                double P, dP[3], hP[3][3], lP, glP[3];
                monomial_derivs(a, b, c, d, &P, dP, hP, &lP, glP);
                double M = m[ao];
                double q[ORACLE_NQ];
                q[0] = M * P * g0;
                for (int x = 0; x < 3; ++x) q[1 + x] = M * (dP[x] * g0 + 2.0 * d[x] * P * g1);
                q[4] = M * (lP * g0 + (4.0 * l + 6.0) * P * g1 + 4.0 * u * P * g2);
                if (nq == ORACLE_NQ) {
                    int hq = 5;
                    for (int x = 0; x < 3; ++x)
                        for (int y = x; y < 3; ++y) {
                            double h = hP[x][y] * g0 + 2.0 * (d[y] * dP[x] + d[x] * dP[y]) * g1 +
                                       4.0 * d[x] * d[y] * P * g2;
                            if (x == y) h += 2.0 * P * g1;
                            q[hq++] = M * h;
                        }
                    for (int x = 0; x < 3; ++x)
                        q[11 + x] = M * (glP[x] * g0 + (2.0 * d[x] * lP + (4.0 * l + 6.0) * dP[x]) * g1 +
                                         ((8.0 * l + 20.0) * d[x] * P + 4.0 * u * dP[x]) * g2 +
                                         8.0 * u * d[x] * P * g3);
                }
                for (int qq = 0; qq < nq; ++qq) o[(size_t)qq * (size_t)ao_num + (size_t)ao] = q[qq];
            }
        }
    }
    free(f);
    free(ns);
    free(m);
    return 0;
}

/*
 * MO contraction (Section 3.2): mo[p][c][n] = sum_k C[n][k] ao[p][c][k] for
 * the five components c, summed sequentially in k.
 */
int oracle_mo_vgl(int64_t point_num, int64_t ao_num, int64_t mo_num, const double* ao,
                  const double* coef, double* mo) {
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < point_num; ++p)
        for (int c = 0; c < 5; ++c) {
            const double* a = ao + ((size_t)p * 5 + (size_t)c) * (size_t)ao_num;
            double* o = mo + ((size_t)p * 5 + (size_t)c) * (size_t)mo_num;
            for (int64_t n = 0; n < mo_num; ++n) {
                const double* cn = coef + (size_t)n * (size_t)ao_num;
                double s = 0.0;
                for (int64_t k = 0; k < ao_num; ++k) s += cn[k] * a[k];
                o[n] = s;
            }
        }
    return 0;
}

/*
 * Adjoint of L = sum_{p,c,n} W[p][c][n] mo[p][c][n] with respect to the MO
 * coefficients, the points and the nuclei (basis parameters fixed, each
 * nucleus carries its shells rigidly):
 *   Gbar[p][c][k] = sum_n W[p][c][n] C[n][k]
 *   dC[n][k]      = sum_{p,c} W[p][c][n] ao[p][c][k]
 *   t[p][k][i]    = Gbar[p][0][k] d_i chi_k + sum_j Gbar[p][1+j][k] d_i d_j chi_k
 *                   + Gbar[p][4][k] d_i lap chi_k
 *   dR_elec[p][i] = sum_k t[p][k][i]
 *   dR_nucl[A][i] = - sum_p sum_{k on A} t[p][k][i]   (chi depends on r - R_A)
 * The *_abs outputs hold the same sums over absolute values of the terms
 * (used to scale tolerances); any output pointer may be NULL.
 */
int oracle_adjoint(int64_t nucl_num, const double* nucl_coord, int64_t shell_num,
                   const int64_t* shell_nucleus, const int32_t* shell_ang_mom,
                   const int64_t* shell_prim_offset, const double* exponent,
                   const double* coefficient, int64_t point_num, const double* point, double B,
                   int64_t mo_num, const double* coef, const double* w, double* d_coef,
                   double* d_elec, double* d_nucl, double* d_coef_abs, double* d_elec_abs,
                   double* d_nucl_abs) {
    int64_t ao_num = oracle_ao_num(shell_num, shell_ang_mom);
    size_t per_point = (size_t)ORACLE_NQ * (size_t)ao_num;
    double* ao = (double*)malloc(sizeof(double) * (size_t)(point_num > 0 ? point_num : 1) * per_point);
    double* nuc_part = (double*)calloc((size_t)(point_num > 0 ? point_num : 1) * (size_t)nucl_num * 6, sizeof(double));
    int64_t* ao_nucleus = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ao_num > 0 ? ao_num : 1));
    if (!ao || !nuc_part || !ao_nucleus) { free(ao); free(nuc_part); free(ao_nucleus); return 2; }
    int rc = oracle_ao_derivs(nucl_num, nucl_coord, shell_num, shell_nucleus, shell_ang_mom,
                              shell_prim_offset, exponent, coefficient, point_num, point, B,
                              ORACLE_NQ, ao);
    if (rc) { free(ao); free(nuc_part); free(ao_nucleus); return rc; }
    {
        int64_t k = 0;
        for (int64_t s = 0; s < shell_num; ++s)
            for (int i = 0; i < n_cart(shell_ang_mom[s]); ++i) ao_nucleus[k++] = shell_nucleus[s];
    }
    /* Hessian quantity index for the (i, j) pair. */
    static const int hidx[3][3] = {{5, 6, 7}, {6, 8, 9}, {7, 9, 10}};

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < point_num; ++p) {
        const double* a = ao + (size_t)p * per_point;
        double de[3] = {0, 0, 0}, dea[3] = {0, 0, 0};
        double* np_ = nuc_part + (size_t)p * (size_t)nucl_num * 6;
        for (int64_t k = 0; k < ao_num; ++k) {
            double gb[5];
            for (int c = 0; c < 5; ++c) {
                double s = 0.0;
                for (int64_t n = 0; n < mo_num; ++n)
                    s += w[((size_t)p * 5 + (size_t)c) * (size_t)mo_num + (size_t)n] *
                         coef[(size_t)n * (size_t)ao_num + (size_t)k];
                gb[c] = s;
            }
            for (int i = 0; i < 3; ++i) {
                double terms[5];
                terms[0] = gb[0] * a[(size_t)(1 + i) * (size_t)ao_num + (size_t)k];
                for (int j = 0; j < 3; ++j)
                    terms[1 + j] = gb[1 + j] * a[(size_t)hidx[i][j] * (size_t)ao_num + (size_t)k];
                terms[4] = gb[4] * a[(size_t)(11 + i) * (size_t)ao_num + (size_t)k];
                double t = 0.0, ta = 0.0;
                for (int q = 0; q < 5; ++q) { t += terms[q]; ta += fabs(terms[q]); }
                de[i] += t;
                dea[i] += ta;
                np_[ao_nucleus[k] * 6 + i] -= t;
                np_[ao_nucleus[k] * 6 + 3 + i] += ta;
            }
        }
        for (int i = 0; i < 3; ++i) {
            if (d_elec) d_elec[3 * p + i] = de[i];
            if (d_elec_abs) d_elec_abs[3 * p + i] = dea[i];
        }
    }
    if (d_nucl || d_nucl_abs) {
        for (int64_t A = 0; A < nucl_num; ++A)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0, sa = 0.0;
                for (int64_t p = 0; p < point_num; ++p) {
                    s += nuc_part[((size_t)p * (size_t)nucl_num + (size_t)A) * 6 + (size_t)i];
                    sa += nuc_part[((size_t)p * (size_t)nucl_num + (size_t)A) * 6 + 3 + (size_t)i];
                }
                if (d_nucl) d_nucl[3 * A + i] = s;
                if (d_nucl_abs) d_nucl_abs[3 * A + i] = sa;
            }
    }
    if (d_coef || d_coef_abs) {
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < mo_num; ++n)
            for (int64_t k = 0; k < ao_num; ++k) {
                double s = 0.0, sa = 0.0;
                for (int64_t p = 0; p < point_num; ++p)
                    for (int c = 0; c < 5; ++c) {
                        double t = w[((size_t)p * 5 + (size_t)c) * (size_t)mo_num + (size_t)n] *
                                   ao[(size_t)p * per_point + (size_t)c * (size_t)ao_num + (size_t)k];
                        s += t;
                        sa += fabs(t);
                    }
                if (d_coef) d_coef[(size_t)n * (size_t)ao_num + (size_t)k] = s;
                if (d_coef_abs) d_coef_abs[(size_t)n * (size_t)ao_num + (size_t)k] = sa;
            }
    }
    free(ao);
    free(nuc_part);
    free(ao_nucleus);
    return 0;
}
