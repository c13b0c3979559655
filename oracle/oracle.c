/*
 * CPU oracle for the multi-determinant evaluation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no code, header or generated table with the GPU
 * library; the two meet only in the seeded input arrays.
 *
 * Everything here is the plain definition, in FP64, with no table, no
 * Sherman-Morrison update and no determinant lemma:
 *
 *   Psi = sum_I c_I det M_up,I det M_dn,I                     (Sec. II, Psi eq.)
 *   M_sigma,I(i,j) = phi_{col(j)}(r_i)                           (Sec. II, M eq.)
 *
 * where the column list col() of a determinant is the reference list 0..n-1
 * with hole h_j replaced in place by particle p_j (particle-hole excitation,
 * Sec. II).  Every determinant is computed by LU with partial pivoting of the
 * full n x n matrix, in the log domain (sign, log|det|).
 *
 * Derivatives for electron i (Sec. IV, eqs. gradMDS and gradDet0): the
 * determinant is linear in row i, the only row that depends on r_i, so
 * grad_i^a det M = det(M with row i replaced by grad^a of that row), for
 * a = x, y, z and for the laplacian alike.  The oracle forms that matrix and
 * takes a second full LU.
 *
 * Adjoint: d det X / dX(r,c) = det X (X^-1)(c,r) (Jacobi's formula), applied
 * to full n x n matrices and their explicit inverses.
 *
 * Orbitals: unnormalised s-Gaussians chi_b(r) = exp(-a_b |r - R_b|^2) and
 * molecular orbitals phi_p = sum_b mo[p][b] chi_b, with the closed forms
 *   grad chi = -2 a (r - R) chi,   lap chi = (4 a^2 |r - R|^2 - 6 a) chi.
 *
 * One function at the end (oracle_mixed_scales_batch) is a measuring tool
 * rather than a definition: it forms the tables of Sec. III explicitly to
 * bound how far FP32 storage of their entries can move each output.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 128

/* ------------------------------------------------------------------------ */
/* orbitals                                                                  */
/* ------------------------------------------------------------------------ */

/* out[q][c][p], c = 0 value, 1..3 d/dx,d/dy,d/dz, 4 laplacian. */
int oracle_orbitals(int nb, const double *centres, const double *expo,
                    int n_orb, const double *mo, int npos, const double *pos,
                    double *out)
{
    double *chi = (double *)malloc(sizeof(double) * 5 * (size_t)nb);
    if (!chi) return -1;
    for (int q = 0; q < npos; ++q) {
        const double *r = pos + 3 * (size_t)q;
        for (int b = 0; b < nb; ++b) {
            double dx = r[0] - centres[3 * b + 0];
            double dy = r[1] - centres[3 * b + 1];
            double dz = r[2] - centres[3 * b + 2];
            double a = expo[b];
            double r2 = dx * dx + dy * dy + dz * dz;
            double v = exp(-a * r2);
            chi[5 * b + 0] = v;
            chi[5 * b + 1] = -2.0 * a * dx * v;
            chi[5 * b + 2] = -2.0 * a * dy * v;
            chi[5 * b + 3] = -2.0 * a * dz * v;
            chi[5 * b + 4] = (4.0 * a * a * r2 - 6.0 * a) * v;
        }
        double *o = out + (size_t)q * 5 * n_orb;
        for (int p = 0; p < n_orb; ++p) {
            double acc[5] = {0, 0, 0, 0, 0};
            for (int b = 0; b < nb; ++b) {
                double w = mo[(size_t)p * nb + b];
                for (int c = 0; c < 5; ++c) acc[c] += w * chi[5 * b + c];
            }
            for (int c = 0; c < 5; ++c) o[(size_t)c * n_orb + p] = acc[c];
        }
    }
    free(chi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* dense linear algebra                                                      */
/* ------------------------------------------------------------------------ */

/* In-place LU with partial pivoting (Doolittle).  a is n x n row-major.
 * perm[k] = row swapped with row k at step k.  Returns the determinant as
 * (sign, log|det|); an exactly zero pivot gives sign 0, log -inf. */
static void lu_factor(int n, double *a, int *perm, double *sign, double *logabs)
{
    double s = 1.0, l = 0.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(a[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        perm[k] = p;
        if (best == 0.0) {
            *sign = 0.0;
            *logabs = -INFINITY;
            for (int kk = k + 1; kk < n; ++kk) perm[kk] = kk;
            return;
        }
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[k * n + j];
                a[k * n + j] = a[p * n + j];
                a[p * n + j] = t;
            }
            s = -s;
        }
        double piv = a[k * n + k];
        if (piv < 0.0) s = -s;
        l += log(fabs(piv));
        for (int i = k + 1; i < n; ++i) {
            double f = a[i * n + k] / piv;
            a[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= f * a[k * n + j];
        }
    }
    *sign = s;
    *logabs = l;
}

int oracle_slogdet(int n, const double *m, double *sign, double *logabs)
{
    if (n <= 0) { *sign = 1.0; *logabs = 0.0; return 0; }
    if (n > OR_MAXN) return -1;
    double a[OR_MAXN * OR_MAXN];
    int perm[OR_MAXN];
    memcpy(a, m, sizeof(double) * (size_t)n * n);
    lu_factor(n, a, perm, sign, logabs);
    return 0;
}

/* Explicit inverse from the LU factors: solve A x = e_c for every c. */
static int lu_inverse(int n, const double *lu, const int *perm, double *inv)
{
    double col[OR_MAXN];
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < n; ++k) {          /* apply the row swaps */
            int p = perm[k];
            if (p != k) { double t = col[k]; col[k] = col[p]; col[p] = t; }
        }
        for (int i = 0; i < n; ++i)            /* forward, unit lower */
            for (int k = 0; k < i; ++k) col[i] -= lu[i * n + k] * col[k];
        for (int i = n - 1; i >= 0; --i) {     /* backward, upper */
            for (int k = i + 1; k < n; ++k) col[i] -= lu[i * n + k] * col[k];
            col[i] /= lu[i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[i * n + c] = col[i];
    }
    return 0;
}

int oracle_inverse(int n, const double *m, double *inv, double *sign, double *logabs)
{
    if (n > OR_MAXN) return -1;
    double a[OR_MAXN * OR_MAXN];
    int perm[OR_MAXN];
    memcpy(a, m, sizeof(double) * (size_t)n * n);
    lu_factor(n, a, perm, sign, logabs);
    if (*sign == 0.0) return 1;
    return lu_inverse(n, a, perm, inv);
}

/* ------------------------------------------------------------------------ */
/* excited matrices                                                          */
/* ------------------------------------------------------------------------ */

/* Column list of excitation u: reference 0..n-1, hole h_j -> particle p_j. */
static void exc_columns(int n, const int *off, const int *hs, const int *ps, int u,
                        int *col)
{
    for (int j = 0; j < n; ++j) col[j] = j;
    for (int t = off[u]; t < off[u + 1]; ++t) col[hs[t]] = ps[t];
}

/* M[i][j] = orb[i][comp_i][col[j]], comp_i = 0 except row `row_d` which takes
 * component `comp` (derivative row replacement). */
static void build_matrix(int n, int n_orb, const double *orb, const int *col,
                         int row_d, int comp, double *M)
{
    for (int i = 0; i < n; ++i) {
        int c = (i == row_d) ? comp : 0;
        const double *r = orb + ((size_t)i * 5 + c) * n_orb;
        for (int j = 0; j < n; ++j) M[i * n + j] = r[col[j]];
    }
}

/* ------------------------------------------------------------------------ */
/* Psi, ratios, derivatives for one walker                                   */
/* ------------------------------------------------------------------------ */

/* out[0] shift used, out[1] psi = sum_I c_I D_up D_dn exp(-shift),
 * out[2..5] the same sum with the moved electron's row replaced by
 * d/dx, d/dy, d/dz, laplacian (zero when e_deriv < 0),
 * out[6..9] sign and log|det| of the up and down reference determinants,
 * out[10] sum of |terms| of out[1], out[11..14] sums of |terms| of
 * out[2..5] (scales for condition-aware comparisons).
 * ratio_up[u] = D_u / D_0 for every up excitation (optional), same for down.
 */
static int mds_walker(int n_up, int n_dn, int no_up, int no_dn,
                      const double *orb_up, const double *orb_dn,
                      int nx_up, const int *off_up, const int *h_up, const int *p_up,
                      int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                      int64_t n_det, const double *coef, const int *iu, const int *id,
                      int e_deriv, double shift, double *out,
                      double *ratio_up, double *ratio_dn)
{
    const int nmax = n_up > n_dn ? n_up : n_dn;
    if (nmax > OR_MAXN) return -1;
    double *sg[2], *lg[2], *sga, *lga;
    int nx[2] = {nx_up, nx_dn};
    for (int s = 0; s < 2; ++s) {
        sg[s] = (double *)malloc(sizeof(double) * (size_t)(nx[s] > 0 ? nx[s] : 1));
        lg[s] = (double *)malloc(sizeof(double) * (size_t)(nx[s] > 0 ? nx[s] : 1));
    }
    int ds = (e_deriv < 0) ? -1 : (e_deriv < n_up ? 0 : 1);
    int nxd = ds < 0 ? 1 : nx[ds];
    sga = (double *)malloc(sizeof(double) * 4 * (size_t)nxd);
    lga = (double *)malloc(sizeof(double) * 4 * (size_t)nxd);
    double *M = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    int col[OR_MAXN], perm[OR_MAXN];

    const int n_s[2] = {n_up, n_dn}, no_s[2] = {no_up, no_dn};
    const double *orb_s[2] = {orb_up, orb_dn};
    const int *off_s[2] = {off_up, off_dn}, *h_s[2] = {h_up, h_dn}, *p_s[2] = {p_up, p_dn};

    for (int s = 0; s < 2; ++s) {
        for (int u = 0; u < nx[s]; ++u) {
            exc_columns(n_s[s], off_s[s], h_s[s], p_s[s], u, col);
            build_matrix(n_s[s], no_s[s], orb_s[s], col, -1, 0, M);
            lu_factor(n_s[s], M, perm, &sg[s][u], &lg[s][u]);
            if (ds == s) {
                int row = (s == 0) ? e_deriv : e_deriv - n_up;
                for (int a = 0; a < 4; ++a) {
                    build_matrix(n_s[s], no_s[s], orb_s[s], col, row, a + 1, M);
                    lu_factor(n_s[s], M, perm, &sga[4 * u + a], &lga[4 * u + a]);
                }
            }
        }
    }
    out[6] = sg[0][0]; out[7] = lg[0][0];
    out[8] = sg[1][0]; out[9] = lg[1][0];
    if (isnan(shift)) shift = lg[0][0] + lg[1][0];
    out[0] = shift;

    double psi = 0.0, dpsi[4] = {0, 0, 0, 0}, apsi = 0.0, adpsi[4] = {0, 0, 0, 0};
    for (int64_t I = 0; I < n_det; ++I) {
        int a = iu[I], b = id[I];
        double t = coef[I] * sg[0][a] * sg[1][b] * exp(lg[0][a] + lg[1][b] - shift);
        psi += t;
        apsi += fabs(t);
        if (ds >= 0) {
            int ue = (ds == 0) ? a : b;   /* excitation of the moved spin */
            int uo = (ds == 0) ? b : a;
            for (int k = 0; k < 4; ++k) {
                double td = coef[I] * sga[4 * ue + k] * sg[1 - ds][uo] *
                            exp(lga[4 * ue + k] + lg[1 - ds][uo] - shift);
                dpsi[k] += td;
                adpsi[k] += fabs(td);
            }
        }
    }
    out[1] = psi;
    for (int k = 0; k < 4; ++k) out[2 + k] = dpsi[k];
    out[10] = apsi;
    for (int k = 0; k < 4; ++k) out[11 + k] = adpsi[k];

    double *rat[2] = {ratio_up, ratio_dn};
    for (int s = 0; s < 2; ++s) {
        if (!rat[s]) continue;
        for (int u = 0; u < nx[s]; ++u)
            rat[s][u] = sg[s][u] * sg[s][0] * exp(lg[s][u] - lg[s][0]);
    }
    for (int s = 0; s < 2; ++s) { free(sg[s]); free(lg[s]); }
    free(sga); free(lga); free(M);
    return 0;
}

/* Batched over W walkers (OpenMP over walkers).  Strides: orb_up walker
 * stride n_up*5*no_up etc.  shift[w] may be NaN (use the walker's own
 * reference log-determinants).  out is [W][15]; ratio_* are [W][nx_*] or NULL. */
int oracle_mds_batch(int W, int n_up, int n_dn, int no_up, int no_dn,
                     const double *orb_up, const double *orb_dn,
                     int nx_up, const int *off_up, const int *h_up, const int *p_up,
                     int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                     int64_t n_det, const double *coef, const int *iu, const int *id,
                     int e_deriv, const double *shift, double *out,
                     double *ratio_up, double *ratio_dn)
{
    int err = 0;
    const size_t su = (size_t)n_up * 5 * no_up, sd = (size_t)n_dn * 5 * no_dn;
#pragma omp parallel for schedule(dynamic) reduction(|: err)
    for (int w = 0; w < W; ++w) {
        err |= mds_walker(n_up, n_dn, no_up, no_dn, orb_up + w * su, orb_dn + w * sd,
                          nx_up, off_up, h_up, p_up, nx_dn, off_dn, h_dn, p_dn,
                          n_det, coef, iu, id, e_deriv, shift ? shift[w] : NAN,
                          out + (size_t)w * 15,
                          ratio_up ? ratio_up + (size_t)w * nx_up : NULL,
                          ratio_dn ? ratio_dn + (size_t)w * nx_dn : NULL);
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* adjoint with respect to the orbital matrix (Jacobi's formula)             */
/* ------------------------------------------------------------------------ */

/* For one walker: dlog|Psi| / d Phi_sigma[i][p] for every electron i and
 * orbital p of both spins (values only, no derivative rows), and
 * dlog|Psi|/dc_I.  g_up is [n_up][no_up], g_dn [n_dn][no_dn]. */
int oracle_psi_adjoint(int n_up, int n_dn, int no_up, int no_dn,
                       const double *orb_up, const double *orb_dn,
                       int nx_up, const int *off_up, const int *h_up, const int *p_up,
                       int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                       int64_t n_det, const double *coef, const int *iu, const int *id,
                       double *out2, double *grad_c, double *g_up, double *g_dn)
{
    const int n_s[2] = {n_up, n_dn}, no_s[2] = {no_up, no_dn}, nx[2] = {nx_up, nx_dn};
    const double *orb_s[2] = {orb_up, orb_dn};
    const int *off_s[2] = {off_up, off_dn}, *h_s[2] = {h_up, h_dn}, *p_s[2] = {p_up, p_dn};
    double *g_s[2] = {g_up, g_dn};
    int nmax = n_up > n_dn ? n_up : n_dn;
    if (nmax > OR_MAXN) return -1;
    double *sg[2], *lg[2];
    for (int s = 0; s < 2; ++s) {
        sg[s] = (double *)malloc(sizeof(double) * (size_t)nx[s]);
        lg[s] = (double *)malloc(sizeof(double) * (size_t)nx[s]);
    }
    double *M = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    double *iv = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    int col[OR_MAXN], perm[OR_MAXN];
    for (int s = 0; s < 2; ++s)
        for (int u = 0; u < nx[s]; ++u) {
            exc_columns(n_s[s], off_s[s], h_s[s], p_s[s], u, col);
            build_matrix(n_s[s], no_s[s], orb_s[s], col, -1, 0, M);
            lu_factor(n_s[s], M, perm, &sg[s][u], &lg[s][u]);
        }
    double shift = lg[0][0] + lg[1][0];
    double psi = 0.0;
    for (int64_t I = 0; I < n_det; ++I)
        psi += coef[I] * sg[0][iu[I]] * sg[1][id[I]] *
               exp(lg[0][iu[I]] + lg[1][id[I]] - shift);
    out2[0] = (psi > 0) - (psi < 0);
    out2[1] = log(fabs(psi)) + shift;
    for (int64_t I = 0; I < n_det; ++I)
        grad_c[I] = sg[0][iu[I]] * sg[1][id[I]] *
                    exp(lg[0][iu[I]] + lg[1][id[I]] - shift) / psi;
    /* chain rule term by term: d/dPhi of c_I D_up,I D_dn,I / Psi */
    for (int s = 0; s < 2; ++s) {
        int n = n_s[s], no = no_s[s];
        memset(g_s[s], 0, sizeof(double) * (size_t)n * no);
        for (int64_t I = 0; I < n_det; ++I) {
            int u = (s == 0) ? iu[I] : id[I];
            int o = (s == 0) ? id[I] : iu[I];
            double w = coef[I] * sg[s][u] * sg[1 - s][o] *
                       exp(lg[s][u] + lg[1 - s][o] - shift) / psi;
            if (w == 0.0) continue;
            double s2, l2;
            exc_columns(n, off_s[s], h_s[s], p_s[s], u, col);
            build_matrix(n, no, orb_s[s], col, -1, 0, M);
            lu_factor(n, M, perm, &s2, &l2);
            lu_inverse(n, M, perm, iv);
            /* M(i,j) = Phi[i][col j]:  d det/dM(i,j) = det * inv(j,i) */
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    g_s[s][(size_t)i * no + col[j]] += w * iv[j * n + i];
        }
    }
    for (int s = 0; s < 2; ++s) { free(sg[s]); free(lg[s]); }
    free(M); free(iv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Psi/Psi0 from explicit tables, and its adjoint                            */
/* ------------------------------------------------------------------------ */

/* With T_sigma = [I | T_V,sigma] given explicitly (n x (n+m)), the excited
 * matrix relative to the reference is X_u = I with column h_j replaced by
 * T[:, p_j]; det X_u = D_u / D_0 by definition of T = A^-1 Phi.  The oracle
 * takes det X_u by full n x n LU and the adjoint by Jacobi's formula on the
 * explicit inverse of X_u.
 *   N = sum_I c_I det X_up,I det X_dn,I
 * out2 = (sign N, log|N|); grad_c[I] = dlog|N|/dc_I;
 * gT_sigma[r][p - n] = dlog|N| / dT_V,sigma[r][p]. */
static void table_matrix(int n, int m, const double *T, const int *off, const int *hs,
                         const int *ps, int u, double *X)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) X[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int t = off[u]; t < off[u + 1]; ++t) {
        int h = hs[t], p = ps[t] - n;
        for (int i = 0; i < n; ++i) X[i * n + h] = T[(size_t)i * m + p];
    }
}

static int tables_walker(int n_up, int n_dn, int m_up, int m_dn,
                         const double *T_up, const double *T_dn,
                         int nx_up, const int *off_up, const int *h_up, const int *p_up,
                         int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                         int64_t n_det, const double *coef, const int *iu, const int *id,
                         double *out2, double *grad_c, double *gT_up, double *gT_dn)
{
    const int n_s[2] = {n_up, n_dn}, m_s[2] = {m_up, m_dn}, nx[2] = {nx_up, nx_dn};
    const double *T_s[2] = {T_up, T_dn};
    const int *off_s[2] = {off_up, off_dn}, *h_s[2] = {h_up, h_dn}, *p_s[2] = {p_up, p_dn};
    double *gT_s[2] = {gT_up, gT_dn};
    int nmax = n_up > n_dn ? n_up : n_dn;
    if (nmax > OR_MAXN) return -1;
    double *val[2];
    for (int s = 0; s < 2; ++s) val[s] = (double *)malloc(sizeof(double) * (size_t)nx[s]);
    double *X = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    double *iv = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    int perm[OR_MAXN];
    for (int s = 0; s < 2; ++s)
        for (int u = 0; u < nx[s]; ++u) {
            double sg, lg;
            table_matrix(n_s[s], m_s[s], T_s[s], off_s[s], h_s[s], p_s[s], u, X);
            lu_factor(n_s[s], X, perm, &sg, &lg);
            val[s][u] = sg * exp(lg);
        }
    double N = 0.0;
    for (int64_t I = 0; I < n_det; ++I) N += coef[I] * val[0][iu[I]] * val[1][id[I]];
    out2[0] = (N > 0) - (N < 0);
    out2[1] = log(fabs(N));
    for (int64_t I = 0; I < n_det; ++I) grad_c[I] = val[0][iu[I]] * val[1][id[I]] / N;
    /* chain rule term by term: d/dT of c_I det X_up,I det X_dn,I / N */
    for (int s = 0; s < 2; ++s) {
        int n = n_s[s], m = m_s[s];
        memset(gT_s[s], 0, sizeof(double) * (size_t)n * m);
        for (int64_t I = 0; I < n_det; ++I) {
            int u = (s == 0) ? iu[I] : id[I];
            int o = (s == 0) ? id[I] : iu[I];
            double w = coef[I] * val[1 - s][o] / N;
            if (w == 0.0 || off_s[s][u + 1] == off_s[s][u]) continue;
            double sg, lg;
            table_matrix(n, m, T_s[s], off_s[s], h_s[s], p_s[s], u, X);
            lu_factor(n, X, perm, &sg, &lg);
            if (sg == 0.0) {
                /* singular X: fall back to cofactors by column replacement,
                 * cof(r,h) = det(X with column h -> e_r) */
                for (int t = off_s[s][u]; t < off_s[s][u + 1]; ++t) {
                    int h = h_s[s][t], p = p_s[s][t] - n;
                    for (int r = 0; r < n; ++r) {
                        double s3, l3;
                        table_matrix(n, m, T_s[s], off_s[s], h_s[s], p_s[s], u, X);
                        for (int i = 0; i < n; ++i) X[i * n + h] = (i == r) ? 1.0 : 0.0;
                        lu_factor(n, X, perm, &s3, &l3);
                        gT_s[s][(size_t)r * m + p] += w * s3 * exp(l3);
                    }
                }
                continue;
            }
            lu_inverse(n, X, perm, iv);
            double d = sg * exp(lg);
            /* X(r, h_j) = T(r, p_j):  d det X / d X(r,h) = det X inv(h, r) */
            for (int t = off_s[s][u]; t < off_s[s][u + 1]; ++t) {
                int h = h_s[s][t], p = p_s[s][t] - n;
                for (int r = 0; r < n; ++r)
                    gT_s[s][(size_t)r * m + p] += w * d * iv[h * n + r];
            }
        }
    }
    for (int s = 0; s < 2; ++s) free(val[s]);
    free(X); free(iv);
    return 0;
}

int oracle_tables_batch(int W, int n_up, int n_dn, int m_up, int m_dn,
                        const double *T_up, const double *T_dn,
                        int nx_up, const int *off_up, const int *h_up, const int *p_up,
                        int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                        int64_t n_det, const double *coef, const int *iu, const int *id,
                        double *out2, double *grad_c, double *gT_up, double *gT_dn)
{
    int err = 0;
    const size_t su = (size_t)n_up * m_up, sd = (size_t)n_dn * m_dn;
#pragma omp parallel for schedule(dynamic) reduction(|: err)
    for (int w = 0; w < W; ++w)
        err |= tables_walker(n_up, n_dn, m_up, m_dn, T_up + w * su, T_dn + w * sd,
                             nx_up, off_up, h_up, p_up, nx_dn, off_dn, h_dn, p_dn,
                             n_det, coef, iu, id, out2 + 2 * (size_t)w,
                             grad_c + (size_t)w * n_det,
                             gT_up + w * su, gT_dn + w * sd);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* first-order error scales of the forms that keep tables in FP32           */
/* (a measuring tool for the parity tests, not part of the values above)    */
/* ------------------------------------------------------------------------ */
/*
 * Table T = A^-1 Phi (Sec. III, table definition); an excitation's ratio is
 * det S with S[j][l] = T[h_j][p_l] (Sec. III read-off).  If every entry is
 * perturbed by |dS_jl| <= eps E_jl, det S moves by at most
 *     eps P_E(S),   P_E(S) = sum_jl E_jl |cof(S)_jl|,   cof = d det S / d S_jl
 * to first order.  E = |S| for entries stored in FP32 (rounding), and
 * E = (|A^-1| |Phi_V|)[h_j][p_l] for entries formed by an FP32 product of
 * A^-1 and Phi_V (a matrix product's error is bounded entrywise by a
 * multiple of the product of the absolute values).
 *
 * Derivatives of the moved electron i at R' (Sec. IV-A): with c' = A'^-1 e_i,
 * rho^a = d^a_O . c' and g^a = d^a_V - d^a_O^T T' (d^a = grad^a of the new
 * orbital row), grad^a D_u(R') / D_0(R') is the bordered determinant
 *     det [[rho^a, -g^a[p]^T], [c'[h], S'_u]]
 * (row replacement read through the determinant lemma); its entries other
 * than rho^a carry FP32 storage in those forms: E = |g^a| or
 * |d^a_V| + |d^a_O^T A'^-1| |Phi'_V| (product form), |c'|, and E of S'.
 *
 * For x = sum_I a_I / sum_I b_I with a_I, b_I products of the two spins'
 * determinants (ratio = rho N'/N, grad^a = A^a / N'), first order gives
 * |dx| <= eps X with
 *   Q(N)  = sum_I |c_I| (P(S_up,I) |R_dn,I| + |R_up,I| P(S_dn,I))
 *   ratio: X = |x| (Q(N')/|N'| + Q(N)/|N|)
 *   grad^a: X = (Q(A^a) + |x| Q(N')) / |N'|
 * out[w][kind][5] = X for (ratio, d/dx, d/dy, d/dz, laplacian), kind 0:
 * rounding of the entries, kind 1: product-formed entries.  vals[w][5] = the
 * same outputs computed by this table route (pinned against the full-LU
 * route of oracle_mds_batch).
 *
 * Tables kept in FP32 across commits (the table update T' = T - c' q^T,
 * q = a'^T T - phi'_V, applied to the stored T, Sec. III) carry the errors of
 * earlier updates: an error dT of the stored table reaches T' as
 * (I - c' a'^T) dT, c' = A'^-1 e_i.  With err_ms [n][m] and err_os the
 * entrywise error magnitudes (in units of eps) of the stored tables of the
 * moving and the other spin (NULL: one rounding, |T|), kind 0 uses E = err
 * for the tables at R and E' = |I - c' a'^T| err_ms + |T'| for T', and
 * err_out [n][m] receives E' (the stored table's magnitudes after a commit).
 */

/* det and cofactor matrix of a k x k matrix (row-major) by LU of each minor */
static double det_cof(int k, const double *M, double *cof)
{
    double a[81], s1, l1;
    int perm[9];
    if (k == 1) { cof[0] = 1.0; return M[0]; }
    for (int j = 0; j < k; ++j)
        for (int l = 0; l < k; ++l) {
            int r = 0;
            for (int jj = 0; jj < k; ++jj) {
                if (jj == j) continue;
                int c = 0;
                for (int ll = 0; ll < k; ++ll) {
                    if (ll == l) continue;
                    a[r * (k - 1) + c] = M[jj * k + ll];
                    ++c;
                }
                ++r;
            }
            lu_factor(k - 1, a, perm, &s1, &l1);
            cof[j * k + l] = (((j + l) & 1) ? -1.0 : 1.0) * s1 * exp(l1);
        }
    double d = 0.0;
    for (int l = 0; l < k; ++l) d += M[l] * cof[l];
    return d;
}

/* inverse, table and product scale of one spin: phi [n][no] values */
static int spin_tables(int n, int no, const double *phi, double *B, double *T, double *E,
                       double *sign, double *logabs)
{
    double A[OR_MAXN * OR_MAXN];
    int perm[OR_MAXN];
    const int m = no - n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[i * n + j] = phi[(size_t)i * no + j];
    lu_factor(n, A, perm, sign, logabs);
    if (*sign == 0.0) return 1;
    lu_inverse(n, A, perm, B);
    for (int r = 0; r < n; ++r)
        for (int p = 0; p < m; ++p) {
            double t = 0.0, e = 0.0;
            for (int k = 0; k < n; ++k) {
                t += B[r * n + k] * phi[(size_t)k * no + n + p];
                e += fabs(B[r * n + k]) * fabs(phi[(size_t)k * no + n + p]);
            }
            T[(size_t)r * m + p] = t;
            E[(size_t)r * m + p] = e;
        }
    return 0;
}

/* ratio of every excitation of one spin from its table, and P_E of it for
 * two entry-magnitude arrays E0 and E1 */
static void spin_ratios(int n, int m, const double *T, const double *E0, const double *E1, int nx,
                        const int *off, const int *hs, const int *ps, double *R, double *P,
                        double *PE)
{
    double S[81], cof[81];
    for (int u = 0; u < nx; ++u) {
        const int k = off[u + 1] - off[u];
        if (k == 0) { R[u] = 1.0; P[u] = 0.0; PE[u] = 0.0; continue; }
        const int *h = hs + off[u], *p = ps + off[u];
        for (int j = 0; j < k; ++j)
            for (int l = 0; l < k; ++l) S[j * k + l] = T[(size_t)h[j] * m + p[l] - n];
        R[u] = det_cof(k, S, cof);
        double a = 0.0, b = 0.0;
        for (int j = 0; j < k; ++j)
            for (int l = 0; l < k; ++l) {
                a += E0[(size_t)h[j] * m + p[l] - n] * fabs(cof[j * k + l]);
                b += E1[(size_t)h[j] * m + p[l] - n] * fabs(cof[j * k + l]);
            }
        P[u] = a;
        PE[u] = b;
    }
}

/* kind-0 error magnitudes of a stored table: given ones, or |T| */
static void err_or_abs(int n, int m, const double *given, const double *T, double *E)
{
    for (size_t q = 0; q < (size_t)n * m; ++q) E[q] = given ? given[q] : fabs(T[q]);
}

static int mixed_walker(int n_up, int n_dn, int no_up, int no_dn, const double *orb_up,
                        const double *orb_dn, int e, const double *blk,
                        int nx_up, const int *off_up, const int *h_up, const int *p_up,
                        int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                        int64_t n_det, const double *coef, const int *iu, const int *id,
                        const double *err_ms, const double *err_os, double *err_out,
                        double *out, double *vals)
{
    const int ms = e < n_up ? 0 : 1, os = 1 - ms;
    const int n_s[2] = {n_up, n_dn}, no_s[2] = {no_up, no_dn}, nx[2] = {nx_up, nx_dn};
    const double *orb_s[2] = {orb_up, orb_dn};
    const int *off_s[2] = {off_up, off_dn}, *h_s[2] = {h_up, h_dn}, *p_s[2] = {p_up, p_dn};
    const int n = n_s[ms], no = no_s[ms], m = no - n, row = ms == 0 ? e : e - n_up;
    const int no2 = no_s[os], n2 = n_s[os], m2 = no2 - n2;
    for (int q = 0; q < 10; ++q) out[q] = NAN;
    for (int q = 0; q < 5; ++q) vals[q] = NAN;
    int nmax = n > n2 ? n : n2, mmax = m > m2 ? m : m2;
    double *phi = malloc(sizeof(double) * (size_t)nmax * (nmax + mmax));
    double *phi2 = malloc(sizeof(double) * (size_t)nmax * (nmax + mmax));
    double *B = malloc(sizeof(double) * (size_t)nmax * nmax);
    double *Bp = malloc(sizeof(double) * (size_t)nmax * nmax);
    double *T = malloc(sizeof(double) * (size_t)nmax * mmax), *E = malloc(sizeof(double) * (size_t)nmax * mmax);
    double *Tp = malloc(sizeof(double) * (size_t)nmax * mmax), *Ep = malloc(sizeof(double) * (size_t)nmax * mmax);
    double *To = malloc(sizeof(double) * (size_t)nmax * mmax), *Eo = malloc(sizeof(double) * (size_t)nmax * mmax);
    double *R = malloc(sizeof(double) * nx[ms] * 3), *Rp = malloc(sizeof(double) * nx[ms] * 3);
    double *Ro = malloc(sizeof(double) * nx[os] * 3);
    double *G = malloc(sizeof(double) * nx[ms] * 12);
    int rc = 0;
    /* moving spin at R and at R' (row `row` replaced), other spin at R */
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < no; ++p) {
            phi[(size_t)i * no + p] = orb_s[ms][((size_t)i * 5) * no + p];
            phi2[(size_t)i * no + p] = i == row ? blk[p] : phi[(size_t)i * no + p];
        }
    double s0, l0, s1, l1, so, lo;
    rc |= spin_tables(n, no, phi, B, T, E, &s0, &l0);
    rc |= spin_tables(n, no, phi2, Bp, Tp, Ep, &s1, &l1);
    {
        double *ph = malloc(sizeof(double) * (size_t)n2 * no2);
        for (int i = 0; i < n2; ++i)
            for (int p = 0; p < no2; ++p) ph[(size_t)i * no2 + p] = orb_s[os][((size_t)i * 5) * no2 + p];
        rc |= spin_tables(n2, no2, ph, B, To, Eo, &so, &lo);   /* B reused as scratch */
        free(ph);
        /* restore B of the moving spin at R (not needed further) */
    }
    double *K0 = malloc(sizeof(double) * (size_t)nmax * mmax);    /* kind 0, moving spin at R */
    double *K0p = malloc(sizeof(double) * (size_t)nmax * mmax);   /* kind 0, T' */
    double *K0o = malloc(sizeof(double) * (size_t)nmax * mmax);   /* kind 0, other spin */
    double cp[OR_MAXN];
    if (rc == 0) {
        for (int r = 0; r < n; ++r) cp[r] = Bp[r * n + row];
        err_or_abs(n, m, err_ms, T, K0);
        err_or_abs(n2, m2, err_os, To, K0o);
        /* T' inherits the stored table's errors through I - c' a'^T */
        for (int r = 0; r < n; ++r)
            for (int p = 0; p < m; ++p) {
                double acc = fabs(Tp[(size_t)r * m + p]);
                for (int k = 0; k < n; ++k) {
                    const double pr = fabs((r == k ? 1.0 : 0.0) - cp[r] * phi2[(size_t)row * no + k]);
                    acc += pr * K0[(size_t)k * m + p];
                }
                K0p[(size_t)r * m + p] = acc;
            }
        if (err_out) memcpy(err_out, K0p, sizeof(double) * (size_t)n * m);
        spin_ratios(n, m, T, K0, E, nx[ms], off_s[ms], h_s[ms], p_s[ms], R, R + nx[ms], R + 2 * nx[ms]);
        spin_ratios(n, m, Tp, K0p, Ep, nx[ms], off_s[ms], h_s[ms], p_s[ms], Rp, Rp + nx[ms], Rp + 2 * nx[ms]);
        spin_ratios(n2, m2, To, K0o, Eo, nx[os], off_s[os], h_s[os], p_s[os], Ro, Ro + nx[os], Ro + 2 * nx[os]);
        /* derivative factors at R' */
        double rho[4], g[4][256], Eg[4][256], Eg0[4][256];
        for (int a = 0; a < 4; ++a) {
            const double *d = blk + (size_t)(1 + a) * no;
            double ra = 0.0, ea[OR_MAXN];
            for (int r = 0; r < n; ++r) ra += d[r] * cp[r];
            rho[a] = ra;
            for (int j = 0; j < n; ++j) {
                double t = 0.0;
                for (int r = 0; r < n; ++r) t += d[r] * Bp[r * n + j];
                ea[j] = t;
            }
            for (int p = 0; p < m; ++p) {
                double t = d[n + p], ee = 0.0;
                for (int r = 0; r < n; ++r) {
                    t -= d[r] * Tp[(size_t)r * m + p];
                    ee += fabs(ea[r]) * fabs(phi2[(size_t)r * no + n + p]);
                }
                g[a][p] = t;
                Eg[a][p] = fabs(d[n + p]) + ee;
                /* g^a = d^a_V - d^a_O^T T' carries the stored table's error */
                double e0 = fabs(t);
                for (int r = 0; r < n; ++r) e0 += fabs(d[r]) * K0p[(size_t)r * m + p];
                Eg0[a][p] = e0;
            }
        }
        /* bordered determinants per excitation of the moving spin */
        double Bo[100], cof[100];
        for (int u = 0; u < nx[ms]; ++u) {
            const int k = off_s[ms][u + 1] - off_s[ms][u];
            const int *h = h_s[ms] + off_s[ms][u], *p = p_s[ms] + off_s[ms][u];
            const int K = k + 1;
            for (int a = 0; a < 4; ++a) {
                Bo[0] = rho[a];
                for (int l = 0; l < k; ++l) Bo[1 + l] = -g[a][p[l] - n];
                for (int j = 0; j < k; ++j) {
                    Bo[(1 + j) * K] = cp[h[j]];
                    for (int l = 0; l < k; ++l) Bo[(1 + j) * K + 1 + l] = Tp[(size_t)h[j] * m + p[l] - n];
                }
                const double d = det_cof(K, Bo, cof);
                double pa = 0.0, pb = 0.0;
                for (int l = 0; l < k; ++l) {
                    pa += Eg0[a][p[l] - n] * fabs(cof[1 + l]);
                    pb += Eg[a][p[l] - n] * fabs(cof[1 + l]);
                }
                for (int j = 0; j < k; ++j) {
                    const double cc = fabs(cp[h[j]]) * fabs(cof[(1 + j) * K]);
                    pa += cc;
                    pb += cc;
                    for (int l = 0; l < k; ++l) {
                        const double cf = fabs(cof[(1 + j) * K + 1 + l]);
                        pa += K0p[(size_t)h[j] * m + p[l] - n] * cf;
                        pb += Ep[(size_t)h[j] * m + p[l] - n] * cf;
                    }
                }
                G[(size_t)u * 12 + a] = d;
                G[(size_t)u * 12 + 4 + a] = pa;
                G[(size_t)u * 12 + 8 + a] = pb;
            }
        }
        /* CI sums */
        double N0 = 0, N1 = 0, Q0[2] = {0, 0}, Q1[2] = {0, 0}, A[4] = {0, 0, 0, 0}, QA[2][4];
        for (int a = 0; a < 4; ++a) QA[0][a] = QA[1][a] = 0.0;
        const int nms = nx[ms], nos = nx[os];
        for (int64_t I = 0; I < n_det; ++I) {
            const int um = ms == 0 ? iu[I] : id[I], uo = ms == 0 ? id[I] : iu[I];
            const double c = coef[I], ac = fabs(c);
            const double ro = Ro[uo], aro = fabs(ro);
            N0 += c * R[um] * ro;
            N1 += c * Rp[um] * ro;
            for (int kind = 0; kind < 2; ++kind) {
                const double po = Ro[(1 + kind) * nos + uo];
                Q0[kind] += ac * (R[(1 + kind) * nms + um] * aro + fabs(R[um]) * po);
                Q1[kind] += ac * (Rp[(1 + kind) * nms + um] * aro + fabs(Rp[um]) * po);
                for (int a = 0; a < 4; ++a)
                    QA[kind][a] += ac * (G[(size_t)um * 12 + 4 + 4 * kind + a] * aro +
                                         fabs(G[(size_t)um * 12 + a]) * po);
            }
            for (int a = 0; a < 4; ++a) A[a] += c * G[(size_t)um * 12 + a] * ro;
        }
        const double rho0 = s0 * s1 * exp(l1 - l0);
        const double ratio = rho0 * N1 / N0;
        vals[0] = ratio;
        for (int a = 0; a < 4; ++a) vals[1 + a] = A[a] / N1;
        for (int kind = 0; kind < 2; ++kind) {
            out[kind * 5] = fabs(ratio) * (Q1[kind] / fabs(N1) + Q0[kind] / fabs(N0));
            for (int a = 0; a < 4; ++a)
                out[kind * 5 + 1 + a] = (QA[kind][a] + fabs(vals[1 + a]) * Q1[kind]) / fabs(N1);
        }
    }
    free(phi); free(phi2); free(B); free(Bp); free(T); free(E); free(Tp); free(Ep);
    free(To); free(Eo); free(R); free(Rp); free(Ro); free(G); free(K0); free(K0p); free(K0o);
    return rc ? 1 : 0;
}

int oracle_mixed_scales_batch(int W, int n_up, int n_dn, int no_up, int no_dn,
                              const double *orb_up, const double *orb_dn, int e,
                              const double *blk,
                              int nx_up, const int *off_up, const int *h_up, const int *p_up,
                              int nx_dn, const int *off_dn, const int *h_dn, const int *p_dn,
                              int64_t n_det, const double *coef, const int *iu, const int *id,
                              const double *err_ms, const double *err_os, double *err_out,
                              double *out, double *vals)
{
    int err = 0;
    const size_t su = (size_t)n_up * 5 * no_up, sd = (size_t)n_dn * 5 * no_dn;
    const int ms = e < n_up ? 0 : 1;
    const size_t sb = (size_t)5 * (ms == 0 ? no_up : no_dn);
    const size_t em = ms == 0 ? (size_t)n_up * (no_up - n_up) : (size_t)n_dn * (no_dn - n_dn);
    const size_t eo = ms == 0 ? (size_t)n_dn * (no_dn - n_dn) : (size_t)n_up * (no_up - n_up);
    if (n_up > OR_MAXN || n_dn > OR_MAXN || no_up - n_up > 256 || no_dn - n_dn > 256) return -1;
#pragma omp parallel for schedule(dynamic) reduction(|: err)
    for (int w = 0; w < W; ++w)
        err |= mixed_walker(n_up, n_dn, no_up, no_dn, orb_up + w * su, orb_dn + w * sd, e,
                            blk + w * sb, nx_up, off_up, h_up, p_up, nx_dn, off_dn, h_dn, p_dn,
                            n_det, coef, iu, id, err_ms ? err_ms + w * em : NULL,
                            err_os ? err_os + w * eo : NULL, err_out ? err_out + w * em : NULL,
                            out + (size_t)w * 10, vals + (size_t)w * 5);
    return err ? -1 : 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
