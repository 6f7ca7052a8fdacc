/*
 * Vecchia log-likelihood oracle: plain, slow, FP64 CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against an
 * independent implementation.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What it computes (James & Guinness, "Implementation and Analysis of GPU
 * Algorithms for Vecchia Approximation"):
 *   - the Vecchia factorisation of the Gaussian density into conditionals of
 *     each ordered observation given its (at most m) nearest previously
 *     ordered neighbours (Section 2.1, Eq. 3);
 *   - for each observation i the sums of Algorithm 1 (Section 3): logdet,
 *     ySy, XSX, ySX and their covariance-parameter derivatives dlogdet,
 *     dySy, dXSX, dySX, plus the Fisher-information sum ainfo;
 *   - covariance: exponential / Matern with half-integer smoothness plus a
 *     nugget whose variance is tau2*sigma2 (Section 4.3, Eq. 6).
 *
 * The paper elides the derivative and Fisher steps of Algorithm 1 ("remaining
 * operations").  This oracle writes them in the plain conditional-Gaussian
 * (kriging-weight) form, which is the definition of the quantities:
 *   conditional of y_i given y_s:  mean b^T y_s with b = Sigma_s^{-1} c,
 *   variance v = Sigma_ii - c^T b,  residuals e_y = y_i - b^T y_s,
 *   e_X = X_i - b^T X_s, and for each parameter theta_j
 *     db_j = Sigma_s^{-1} (dc_j - dSigma_s,j b)
 *     dv_j = dSigma_ii,j - 2 dc_j^T b + b^T dSigma_s,j b.
 *   Per observation:
 *     logdet += log v            ySy += e_y^2 / v
 *     XSX    += e_X e_X^T / v    ySX += e_y e_X / v
 *     dlogdet_j += dv_j / v
 *     dySy_j    += 2 e_y de_y / v - e_y^2 dv_j / v^2,   de_y = -db_j^T y_s
 *     dXSX_j    += (de_X e_X^T + e_X de_X^T) / v - e_X e_X^T dv_j / v^2
 *     dySX_j    += (de_y e_X + e_y de_X) / v - e_y e_X dv_j / v^2
 *     ainfo_jk  += dv_j dv_k / (2 v^2) + db_j^T Sigma_s db_k / v
 *   ainfo is the expected information of each conditional density with the
 *   conditioning values drawn from their Gaussian marginal.
 *
 * Sums over observations use Neumaier (compensated) summation.
 *
 * Raw-sum layout (nraw = 2 + p*p + p + P*(2 + p*p + p) + P*P doubles):
 *   [logdet, ySy, XSX[p][p], ySX[p], dlogdet[P], dySy[P], dXSX[P][p][p],
 *    dySX[P][p], ainfo[P][P]]
 *
 * Covariance parameters (P = number of parameters):
 *   family 0, isotropic:   (sigma2, rho, tau2)                     P = 3
 *   family 1, space-time:  (sigma2, rho_space, rho_time, tau2)     P = 4
 *     the first nspace coordinates are scaled by rho_space, the rest by
 *     rho_time:  h^2 = |dz_space|^2/rho_space^2 + |dz_time|^2/rho_time^2.
 *   family 2, anisotropic: (sigma2, rho_1, ..., rho_d, tau2)      P = d + 2
 *     one range per coordinate (Section 4.3, Eq. 6):
 *     h^2 = sum_k (dz_k / rho_k)^2.
 *   Cov(a,b) = sigma2 * (f_nu(h) + tau2 * [a == b]),  h = scaled distance,
 *   f_0.5(h) = exp(-h), f_1.5(h) = (1+h) exp(-h),
 *   f_2.5(h) = (1 + h + h^2/3) exp(-h).
 *
 * NNarray: int32 [n][m+1], 0-based; row i holds i in column 0 and its
 * q = min(i, m) conditioning neighbours in columns 1..q (any order, each
 * < i), -1 in the unused columns.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOTPD (-2)
#define OR_EBADNN (-3)

#define OR_FAMILY_ISO 0
#define OR_FAMILY_SPACETIME 1
#define OR_FAMILY_ANISO 2
#define OR_MAXP 40 /* most covariance parameters of any family */

int oracle_nparms(int family, int d) {
  if (family == OR_FAMILY_ISO) return 3;
  if (family == OR_FAMILY_SPACETIME) return 4;
  if (family == OR_FAMILY_ANISO && d >= 1 && d <= OR_MAXP - 2) return d + 2;
  return -1;
}

int oracle_nraw(int p, int nparms) {
  return 2 + p * p + p + nparms * (2 + p * p + p) + nparms * nparms;
}

/* Matern correlation with half-integer smoothness, as a function of the
 * scaled distance h, and its derivative in h. */
static int matern(double nu, double h, double* f, double* fp) {
  double e = exp(-h);
  if (nu == 0.5) {
    *f = e;
    *fp = -e;
  } else if (nu == 1.5) {
    *f = (1.0 + h) * e;
    *fp = -h * e;
  } else if (nu == 2.5) {
    *f = (1.0 + h + h * h / 3.0) * e;
    *fp = -(h / 3.0) * (1.0 + h) * e;
  } else {
    return OR_EINVAL;
  }
  return OR_OK;
}

/* Covariance between two locations za, zb (d coordinates each) and its
 * derivative with respect to every covariance parameter.  same = 1 when a
 * and b are the same observation (the nugget applies). */
static int cov_pair(int family, double nu, int nspace, int d, const double* covparms,
                    const double* za, const double* zb, int same, double* c, double* dc) {
  int P = oracle_nparms(family, d);
  double sigma2 = covparms[0];
  double tau2 = covparms[P - 1];
  /* range groups: one (isotropic), space and time, or one per coordinate;
   * hg2[g] = squared scaled distance over the coordinates of group g */
  int ngroups = P - 2;
  double hg2[OR_MAXP];
  for (int g = 0; g < ngroups; ++g) hg2[g] = 0.0;
  for (int k = 0; k < d; ++k) {
    int g = (family == OR_FAMILY_ISO) ? 0
            : (family == OR_FAMILY_SPACETIME) ? (k >= nspace ? 1 : 0)
                                               : k;
    double t = (za[k] - zb[k]) / covparms[1 + g];
    hg2[g] += t * t;
  }
  double hh = 0.0;
  for (int g = 0; g < ngroups; ++g) hh += hg2[g];
  double h = sqrt(hh);
  double f, fp;
  if (matern(nu, h, &f, &fp) != OR_OK) return OR_EINVAL;
  *c = sigma2 * (f + (same ? tau2 : 0.0));
  dc[0] = f + (same ? tau2 : 0.0);
  for (int g = 0; g < ngroups; ++g) {
    /* dh/drho_g = -hg2 / (rho_g h), taken as 0 at h = 0 */
    double dh = (h > 0.0) ? -hg2[g] / (covparms[1 + g] * h) : 0.0;
    dc[1 + g] = sigma2 * fp * dh;
  }
  dc[P - 1] = same ? sigma2 : 0.0;
  return OR_OK;
}

/* Covariance matrix S[k][k] of k locations and its derivatives
 * dS[P][k][k]; every index is its own observation. */
int oracle_cov_matrix(int k, int d, const double* locs, int family, double nu, int nspace,
                      const double* covparms, double* S, double* dS) {
  int P = oracle_nparms(family, d);
  if (P < 0 || k < 0 || d < 1) return OR_EINVAL;
  double dc[OR_MAXP];
  for (int a = 0; a < k; ++a) {
    for (int b = 0; b < k; ++b) {
      int st = cov_pair(family, nu, nspace, d, covparms, locs + (size_t)a * d,
                        locs + (size_t)b * d, a == b, &S[(size_t)a * k + b], dc);
      if (st != OR_OK) return st;
      for (int j = 0; j < P; ++j) dS[((size_t)j * k + a) * k + b] = dc[j];
    }
  }
  return OR_OK;
}

/* Textbook Cholesky A = L L^T of a q x q matrix (row-major, lower part of
 * L written into L, upper part zero).  Returns 0, or -1 if a pivot is not
 * positive. */
static int cholesky(int q, const double* A, double* L) {
  for (int r = 0; r < q; ++r) {
    for (int c = 0; c <= r; ++c) {
      double s = A[r * q + c];
      for (int t = 0; t < c; ++t) s -= L[r * q + t] * L[c * q + t];
      if (r == c) {
        if (!(s > 0.0)) return -1;
        L[r * q + r] = sqrt(s);
      } else {
        L[r * q + c] = s / L[c * q + c];
      }
    }
    for (int c = r + 1; c < q; ++c) L[r * q + c] = 0.0;
  }
  return 0;
}

/* Solve (L L^T) x = rhs for x, by forward then backward substitution. */
static void chol_solve(int q, const double* L, const double* rhs, double* x) {
  for (int r = 0; r < q; ++r) {
    double s = rhs[r];
    for (int t = 0; t < r; ++t) s -= L[r * q + t] * x[t];
    x[r] = s / L[r * q + r];
  }
  for (int r = q - 1; r >= 0; --r) {
    double s = x[r];
    for (int t = r + 1; t < q; ++t) s -= L[t * q + r] * x[t];
    x[r] = s / L[r * q + r];
  }
}

/* Neumaier compensated accumulator. */
typedef struct {
  double sum, comp;
} acc_t;

static void acc_add(acc_t* a, double x) {
  double t = a->sum + x;
  if (fabs(a->sum) >= fabs(x))
    a->comp += (a->sum - t) + x;
  else
    a->comp += (x - t) + a->sum;
  a->sum = t;
}

/*
 * Sums of Algorithm 1 over observations i0 <= i < i1 of an n-observation
 * problem.  locs[n][d], NN[n][m+1], y[n], X[n][p] row-major.  raw receives
 * nraw doubles in the layout documented above.  On a failure *bad_i holds
 * the observation at which it was found and the return value is negative.
 */
int oracle_raw_sums(int64_t n, int m, int d, int p, int family, double nu, int nspace,
                    const double* locs, const int32_t* NN, const double* y, const double* X,
                    const double* covparms, int64_t i0, int64_t i1, double* raw,
                    int64_t* bad_i) {
  int P = oracle_nparms(family, d);
  *bad_i = -1;
  if (P < 0 || n < 1 || m < 0 || d < 1 || p < 1 || i0 < 0 || i1 > n || i0 > i1)
    return OR_EINVAL;
  if (family == OR_FAMILY_SPACETIME && (nspace < 1 || nspace >= d)) return OR_EINVAL;
  if (!(nu == 0.5 || nu == 1.5 || nu == 2.5)) return OR_EINVAL;
  int nraw = oracle_nraw(p, P);
  acc_t* acc = (acc_t*)calloc((size_t)nraw, sizeof(acc_t));
  int Q = m; /* largest conditioning set */
  double* Ss = (double*)malloc(sizeof(double) * (size_t)(Q * Q + 1));
  double* Ls = (double*)malloc(sizeof(double) * (size_t)(Q * Q + 1));
  double* dSs = (double*)malloc(sizeof(double) * (size_t)(P * Q * Q + 1));
  double* cvec = (double*)malloc(sizeof(double) * (size_t)(Q + 1));
  double* dcvec = (double*)malloc(sizeof(double) * (size_t)(P * Q + 1));
  double* b = (double*)malloc(sizeof(double) * (size_t)(Q + 1));
  double* db = (double*)malloc(sizeof(double) * (size_t)(P * Q + 1));
  double* tmp = (double*)malloc(sizeof(double) * (size_t)(Q + 1));
  double* eX = (double*)malloc(sizeof(double) * (size_t)p);
  double* deX = (double*)malloc(sizeof(double) * (size_t)(P * p));
  double* dv = (double*)malloc(sizeof(double) * (size_t)P);
  double* dey = (double*)malloc(sizeof(double) * (size_t)P);
  double dcpair[OR_MAXP];
  int status = OR_OK;

  for (int64_t i = i0; i < i1; ++i) {
    const int32_t* row = NN + (size_t)i * (size_t)(m + 1);
    int q = (int)((i < m) ? i : m);
    if (row[0] != (int32_t)i) {
      status = OR_EBADNN;
      *bad_i = i;
      break;
    }
    for (int a = 0; a < q; ++a) {
      if (row[1 + a] < 0 || (int64_t)row[1 + a] >= i) {
        status = OR_EBADNN;
        *bad_i = i;
        break;
      }
    }
    if (status != OR_OK) break;
    const double* zi = locs + (size_t)i * d;

    /* Sigma_s, c = Sigma[s, i], Sigma_ii and their derivatives */
    for (int a = 0; a < q; ++a) {
      const double* za = locs + (size_t)row[1 + a] * d;
      for (int bb = 0; bb < q; ++bb) {
        const double* zb = locs + (size_t)row[1 + bb] * d;
        cov_pair(family, nu, nspace, d, covparms, za, zb, a == bb, &Ss[a * q + bb], dcpair);
        for (int j = 0; j < P; ++j) dSs[(j * q + a) * q + bb] = dcpair[j];
      }
      cov_pair(family, nu, nspace, d, covparms, za, zi, 0, &cvec[a], dcpair);
      for (int j = 0; j < P; ++j) dcvec[j * q + a] = dcpair[j];
    }
    double sii, dsii[OR_MAXP];
    cov_pair(family, nu, nspace, d, covparms, zi, zi, 1, &sii, dsii);

    /* kriging weights b, conditional variance v, residuals */
    if (q > 0 && cholesky(q, Ss, Ls) != 0) {
      status = OR_ENOTPD;
      *bad_i = i;
      break;
    }
    if (q > 0) chol_solve(q, Ls, cvec, b);
    double v = sii;
    for (int a = 0; a < q; ++a) v -= cvec[a] * b[a];
    if (!(v > 0.0)) {
      status = OR_ENOTPD;
      *bad_i = i;
      break;
    }
    double ey = y[i];
    for (int a = 0; a < q; ++a) ey -= b[a] * y[row[1 + a]];
    for (int t = 0; t < p; ++t) {
      eX[t] = X[(size_t)i * p + t];
      for (int a = 0; a < q; ++a) eX[t] -= b[a] * X[(size_t)row[1 + a] * p + t];
    }

    /* parameter derivatives of b and v, and of the residuals */
    for (int j = 0; j < P; ++j) {
      const double* dS = dSs + (size_t)j * q * q;
      const double* dcj = dcvec + (size_t)j * q;
      for (int a = 0; a < q; ++a) {
        double s = dcj[a];
        for (int bb = 0; bb < q; ++bb) s -= dS[a * q + bb] * b[bb];
        tmp[a] = s;
      }
      if (q > 0) chol_solve(q, Ls, tmp, db + (size_t)j * q);
      double dvj = dsii[j];
      for (int a = 0; a < q; ++a) dvj -= 2.0 * dcj[a] * b[a];
      for (int a = 0; a < q; ++a)
        for (int bb = 0; bb < q; ++bb) dvj += b[a] * dS[a * q + bb] * b[bb];
      dv[j] = dvj;
      double s = 0.0;
      for (int a = 0; a < q; ++a) s -= db[j * q + a] * y[row[1 + a]];
      dey[j] = s;
      for (int t = 0; t < p; ++t) {
        double sx = 0.0;
        for (int a = 0; a < q; ++a) sx -= db[j * q + a] * X[(size_t)row[1 + a] * p + t];
        deX[j * p + t] = sx;
      }
    }

    /* accumulate in the documented layout */
    int o = 0;
    acc_add(&acc[o++], log(v));
    acc_add(&acc[o++], ey * ey / v);
    for (int s = 0; s < p; ++s)
      for (int t = 0; t < p; ++t) acc_add(&acc[o++], eX[s] * eX[t] / v);
    for (int t = 0; t < p; ++t) acc_add(&acc[o++], ey * eX[t] / v);
    for (int j = 0; j < P; ++j) acc_add(&acc[o++], dv[j] / v);
    for (int j = 0; j < P; ++j)
      acc_add(&acc[o++], 2.0 * ey * dey[j] / v - ey * ey * dv[j] / (v * v));
    for (int j = 0; j < P; ++j)
      for (int s = 0; s < p; ++s)
        for (int t = 0; t < p; ++t)
          acc_add(&acc[o++], (deX[j * p + s] * eX[t] + eX[s] * deX[j * p + t]) / v -
                                 eX[s] * eX[t] * dv[j] / (v * v));
    for (int j = 0; j < P; ++j)
      for (int t = 0; t < p; ++t)
        acc_add(&acc[o++], (dey[j] * eX[t] + ey * deX[j * p + t]) / v -
                               ey * eX[t] * dv[j] / (v * v));
    for (int j = 0; j < P; ++j) {
      for (int k = 0; k < P; ++k) {
        /* db_j^T Sigma_s db_k */
        double quad = 0.0;
        for (int a = 0; a < q; ++a)
          for (int bb = 0; bb < q; ++bb) quad += db[j * q + a] * Ss[a * q + bb] * db[k * q + bb];
        acc_add(&acc[o++], 0.5 * dv[j] * dv[k] / (v * v) + quad / v);
      }
    }
  }

  for (int e = 0; e < nraw; ++e) raw[e] = acc[e].sum + acc[e].comp;
  free(acc);
  free(Ss);
  free(Ls);
  free(dSs);
  free(cvec);
  free(dcvec);
  free(b);
  free(db);
  free(tmp);
  free(eX);
  free(deX);
  free(dv);
  free(dey);
  return status;
}
