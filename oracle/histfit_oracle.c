/*
 * histfit_oracle.c -- plain, slow, FP64 CPU oracle for the binned
 * histogram-fit objective and its parameter gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and by nothing else.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * What it computes (paper, sec. 4 "Integration and Results", Fig. 2a): a
 * parametric function with parameter vector theta is fitted to a uniformly
 * binned histogram by a gradient-based minimiser; the gradient of the fit
 * objective with respect to theta is what reverse-mode AD supplies
 * (sec. 2 "Background": reverse accumulation suits functions with one output
 * and many inputs).  The oracle writes that gradient out by its plain
 * definition -- the chain rule with closed-form partial derivatives of the
 * model -- rather than by an adjoint sweep:
 *
 *   L(theta)      = sum_i w_i * l(n_i, mu_i(theta))
 *   dL/dtheta_k   = sum_i w_i * dl/dmu(n_i, mu_i) * dmu_i/dtheta_k
 *
 * with mu_i the model at the centre of bin i.  Sums are Neumaier-compensated
 * and visited in bin-index order.  Alongside the sums it returns the
 * condition scales S_0 = sum|w_i l_i| and S_k = sum_i |w_i dl/dmu dmu/dtheta_k|
 * that define the relative tolerances of the parity tests.
 *
 * Models (theta order in brackets):
 *   kind 1  1D: sum of n_gauss amplitude-form Gaussians A exp(-z^2/2),
 *           z = (x-m)/s  [A,m,s per Gaussian], plus a polynomial
 *           sum_j c_j t^j, t = (x - t_shift)/t_scale  [c_0..c_D]; D = -1
 *           means no background.  The amplitude form is the "gaus"
 *           function {Constant, Mean, Sigma} used in Fig. 2a.
 *   kind 2  1D: the same Gaussians plus exp(b0 + b1 t)  [b0,b1].
 *   kind 3  2D: A exp(-Q/2) + c with
 *           Q = (u^2 - 2 rho u v + v^2)/(1-rho^2), u = (x-mx)/sx,
 *           v = (y-my)/sy   [A,mx,my,sx,sy,rho,c]; bins are row-major with
 *           x fastest.
 * Objectives (per bin, n = count, mu = model):
 *   0 Neyman chi-square  l = (n-mu)^2/n for n > 0; empty bins are skipped.
 *   1 Pearson chi-square l = (n-mu)^2/mu; mu <= 0 is a domain error.
 *   2 Poisson, saturated form without the factor 2:
 *           l = mu - n + n ln(n/mu) for n > 0, l = mu for n = 0;
 *           mu <= 0 with n > 0, or mu < 0 with n = 0, is a domain error.
 * A domain error makes that bin's l = +inf and sets status bit 0; the
 * objective is then +inf and not differentiable, so the gradient is NaN.
 * A non-finite theta sets status bit 1.
 *
 * The fitter (or_fit) is a textbook BFGS on the inverse Hessian with a
 * backtracking Armijo line search, stopping on the estimated distance to
 * minimum EDM = g^T H g / 2 (Nocedal & Wright, "Numerical Optimization",
 * ch. 6, with the first-step scaling of their eq. 6.20).  The stopping
 * threshold is max(edm_tol, 4 eps |f|): below a few ulps of the objective a
 * decrease can no longer be verified.  Optionally the first inverse Hessian
 * is the inverse of the expected Hessian (Fisher information, or_fisher) at
 * the start instead of the identity, so the first step is a Gauss-Newton
 * (Fisher scoring) step; the eq. 6.20 scaling is then skipped.
 *
 * Further definitions, each written out where it is defined: the expected
 * Hessian (or_fisher); the bin-average form of the 1D models (the model's
 * integral over each bin divided by its width, selected by
 * or_model.bin_average); bins of any widths (or_nll_grad_edges); and the
 * extended unbinned NLL of single events (or_unbinned).
 *
 * The learned initialiser's network is checked by a separate numpy oracle
 * (mlp.py beside this file): the plain forward and backward passes of a
 * dense GELU network with bfloat16 rounding applied at stated points.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -std=c11 -shared -fPIC
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_NEYMAN = 0, OR_PEARSON = 1, OR_POISSON = 2 };
enum { OR_GAUSS_POLY = 1, OR_GAUSS_EXP = 2, OR_GAUSS2D = 3 };
enum { OR_ST_DOMAIN = 1, OR_ST_NONFINITE = 2 };
enum { OR_MAXP = 32 };

typedef struct {
  int32_t kind;
  int32_t n_gauss;
  int32_t poly_degree;
  int32_t bin_average; /* kinds 1, 2: 1 = mu_i is the bin average of the model */
  double t_shift;
  double t_scale;
} or_model;

/* ---------------------------------------------------------------------- */
/* Neumaier (1974) compensated summation: the improved Kahan-Babuska sum.  */
/* Non-finite terms bypass the compensation so that +inf stays +inf.       */
/* ---------------------------------------------------------------------- */
typedef struct {
  double s;
  double c;
} nsum;

static void nsum_add(nsum* a, double v) {
  if (!isfinite(v) || !isfinite(a->s)) {
    a->s += v;
    return;
  }
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static double nsum_value(const nsum* a) {
  if (!isfinite(a->s)) return a->s;
  return a->s + a->c;
}

double or_neumaier_sum(const double* v, int64_t n) {
  nsum a = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) nsum_add(&a, v[i]);
  return nsum_value(&a);
}

/* ---------------------------------------------------------------------- */
/* Models                                                                  */
/* ---------------------------------------------------------------------- */
int or_nparams(const or_model* m) {
  if (!m) return -1;
  if (m->bin_average && (m->kind == OR_GAUSS2D || m->poly_degree > 3)) return -1;
  switch (m->kind) {
    case OR_GAUSS_POLY:
      if (m->n_gauss < 0 || m->poly_degree < -1) return -1;
      if (m->n_gauss == 0 && m->poly_degree < 0) return -1;
      return 3 * m->n_gauss + (m->poly_degree + 1);
    case OR_GAUSS_EXP:
      if (m->n_gauss < 0) return -1;
      return 3 * m->n_gauss + 2;
    case OR_GAUSS2D:
      return 7;
    default:
      return -1;
  }
}

/* mu(x) for the 1D models and, if dmu != NULL, the partial derivatives
 * dmu/dtheta_k written by their closed forms:
 *   dG/dA = e,  dG/dm = A e (x-m)/s^2,  dG/ds = A e (x-m)^2/s^3,
 *   d(sum c_j t^j)/dc_j = t^j,
 *   d exp(b0+b1 t)/db0 = exp(b0+b1 t),  d/db1 = t exp(b0+b1 t).          */
static double model1d(const or_model* m, const double* th, double x, double* dmu) {
  double mu = 0.0;
  int k = 0;
  for (int g = 0; g < m->n_gauss; ++g, k += 3) {
    double A = th[k], mean = th[k + 1], s = th[k + 2];
    double d = x - mean;
    double e = exp(-(d * d) / (2.0 * s * s));
    mu += A * e;
    if (dmu) {
      dmu[k] = e;
      dmu[k + 1] = A * e * d / (s * s);
      dmu[k + 2] = A * e * d * d / (s * s * s);
    }
  }
  double t = (x - m->t_shift) / m->t_scale;
  if (m->kind == OR_GAUSS_POLY) {
    double tj = 1.0;
    for (int j = 0; j <= m->poly_degree; ++j) {
      mu += th[k + j] * tj;
      if (dmu) dmu[k + j] = tj;
      tj *= t;
    }
  } else {
    double E = exp(th[k] + th[k + 1] * t);
    mu += E;
    if (dmu) {
      dmu[k] = E;
      dmu[k + 1] = t * E;
    }
  }
  return mu;
}

/* mu(x,y) for the correlated 2D Gaussian plus constant, with D = 1-rho^2:
 *   dmu/dA   = e
 *   dmu/dmx  = G (u - rho v) / (D sx)      dmu/dmy = G (v - rho u) / (D sy)
 *   dmu/dsx  = G u (u - rho v) / (D sx)    dmu/dsy = G v (v - rho u) / (D sy)
 *   dmu/drho = G (u v - rho Q) / D         dmu/dc  = 1
 * where e = exp(-Q/2) and G = A e.                                       */
static double model2d(const double* th, double x, double y, double* dmu) {
  double A = th[0], mx = th[1], my = th[2], sx = th[3], sy = th[4], rho = th[5], c = th[6];
  double u = (x - mx) / sx;
  double v = (y - my) / sy;
  double D = 1.0 - rho * rho;
  double Q = (u * u - 2.0 * rho * u * v + v * v) / D;
  double e = exp(-0.5 * Q);
  double G = A * e;
  if (dmu) {
    dmu[0] = e;
    dmu[1] = G * (u - rho * v) / (D * sx);
    dmu[2] = G * (v - rho * u) / (D * sy);
    dmu[3] = G * u * (u - rho * v) / (D * sx);
    dmu[4] = G * v * (v - rho * u) / (D * sy);
    dmu[5] = G * (u * v - rho * Q) / D;
    dmu[6] = 1.0;
  }
  return G + c;
}

/* Bin centre of bin i out of n on [lo, hi]: lo + (i + 1/2) (hi - lo)/n.   */
static double centre(double lo, double hi, int64_t n, int64_t i) {
  double h = (hi - lo) / (double)n;
  return lo + ((double)i + 0.5) * h;
}

/* S(u) = sinh(u)/u and S'(u), from their definition as averages over
 * s in [-1, 1]:  S(u) = (1/2) int e^{u s} ds,  S'(u) = (1/2) int s e^{u s} ds.
 * The average of exp(b0 + b1 t) over [t_c - d, t_c + d] is
 * exp(b0 + b1 t_c) S(b1 d).  For |u| < 1 the two integrals are taken by
 * 16-point Gauss-Legendre quadrature (exact to rounding for these entire
 * integrands: the rule integrates polynomials of degree 31), pairing the
 * nodes +-x so that the sums are of cosh(u x) and x sinh(u x), positive
 * terms with no cancellation; for |u| >= 1 by the closed forms sinh(u)/u and
 * (u cosh u - sinh u)/u^2, which no longer cancel badly there.            */
static double gl_x[8], gl_w[8]; /* positive Gauss-Legendre nodes, weights */

/* Nodes and weights of the 16-point Gauss-Legendre rule on [-1, 1]: the
 * roots of the Legendre polynomial P_16 by Newton's method on the
 * three-term recurrence, w = 2 / ((1 - x^2) P_16'(x)^2).                  */
__attribute__((constructor)) static void gauss_legendre16(void) {
  const int n = 16;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n / 2; ++i) {
    double z = cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) <= 1e-16) break;
    }
    gl_x[i] = z;
    gl_w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static void sinhc(double u, double* S, double* dS) {
  if (fabs(u) < 1.0) {
    double s = 0.0, d = 0.0;
    for (int i = 0; i < 8; ++i) {
      s += gl_w[i] * cosh(u * gl_x[i]);
      d += gl_w[i] * gl_x[i] * sinh(u * gl_x[i]);
    }
    *S = s;
    *dS = d;
  } else {
    *S = sinh(u) / u;
    *dS = (u * cosh(u) - sinh(u)) / (u * u);
  }
}

/* Bin average of the kind-1 model over [a, b] (h = b - a): the integral of
 * the model over the bin divided by the bin width, instead of its value at
 * the centre.  Per Gaussian, with z_x = (x - m)/s and e_x = exp(-z_x^2/2):
 *   mu_g   = A s sqrt(pi/2) [erf(z_b/sqrt 2) - erf(z_a/sqrt 2)] / h
 *   dmu/dA = s sqrt(pi/2) [erf(z_b/sqrt 2) - erf(z_a/sqrt 2)] / h
 *   dmu/dm = A (e_a - e_b) / h
 *   dmu/ds = mu_g / s + A (z_a e_a - z_b e_b) / h
 * Polynomial: the average of t^j over [t_c - d, t_c + d], t_c the bin
 * centre's t and d = h / (2 t_scale), is exactly
 *   1,  t_c,  t_c^2 + d^2/3,  t_c^3 + t_c d^2      (j = 0..3),
 * which is also dmu/dc_j.  Exponential (kind 2): E_c S(b1 d) with
 * E_c = exp(b0 + b1 t_c), S(u) = sinh(u)/u; d/db0 = itself,
 * d/db1 = E_c (t_c S + d S').                                              */
static double model1d_avg(const or_model* m, const double* th, double a, double b, double* dmu) {
  const double h = b - a;
  const double rt = sqrt(0.5 * 3.14159265358979323846), r2 = sqrt(2.0);
  double mu = 0.0;
  int k = 0;
  for (int g = 0; g < m->n_gauss; ++g, k += 3) {
    double A = th[k], mean = th[k + 1], s = th[k + 2];
    double za = (a - mean) / s, zb = (b - mean) / s;
    double ea = exp(-0.5 * za * za), eb = exp(-0.5 * zb * zb);
    double ia = s * rt * (erf(zb / r2) - erf(za / r2)) / h;
    double mg = A * ia;
    mu += mg;
    if (dmu) {
      dmu[k] = ia;
      dmu[k + 1] = A * (ea - eb) / h;
      dmu[k + 2] = mg / s + A * (za * ea - zb * eb) / h;
    }
  }
  double tc = (0.5 * (a + b) - m->t_shift) / m->t_scale;
  double d = 0.5 * h / m->t_scale;
  if (m->kind == OR_GAUSS_EXP) {
    /* average of exp(b0 + b1 t): E_c S(b1 d), E_c = exp(b0 + b1 t_c);
     * d/db0 = itself, d/db1 = E_c (t_c S + d S')                          */
    double Ec = exp(th[k] + th[k + 1] * tc), S, dS;
    sinhc(th[k + 1] * d, &S, &dS);
    mu += Ec * S;
    if (dmu) {
      dmu[k] = Ec * S;
      dmu[k + 1] = Ec * (tc * S + d * dS);
    }
    return mu;
  }
  double avg[4] = {1.0, tc, tc * tc + d * d / 3.0, tc * tc * tc + tc * d * d};
  for (int j = 0; j <= m->poly_degree; ++j) {
    mu += th[k + j] * avg[j];
    if (dmu) dmu[k + j] = avg[j];
  }
  return mu;
}

/* mu of bin i.  edges (1D, nullable): the nx + 1 bin edges of a histogram
 * with bins of any widths; bin i spans [edges[i], edges[i+1]] and its
 * centre is their midpoint.  Without edges the bins are uniform on r.     */
static double eval_mu(const or_model* m, const double* th, int64_t nx, int64_t ny,
                      const double* r, const double* edges, int64_t i, double* dmu) {
  if (m->kind == OR_GAUSS2D) {
    int64_t ix = i % nx, iy = i / nx;
    return model2d(th, centre(r[0], r[1], nx, ix), centre(r[2], r[3], ny, iy), dmu);
  }
  (void)ny;
  if (edges) {
    if (m->bin_average) return model1d_avg(m, th, edges[i], edges[i + 1], dmu);
    return model1d(m, th, 0.5 * (edges[i] + edges[i + 1]), dmu);
  }
  if (m->bin_average) {
    double h = (r[1] - r[0]) / (double)nx;
    return model1d_avg(m, th, r[0] + (double)i * h, r[0] + (double)(i + 1) * h, dmu);
  }
  return model1d(m, th, centre(r[0], r[1], nx, i), dmu);
}

int or_model_eval(const or_model* m, const double* th, int64_t nx, int64_t ny,
                  const double* range4, double* mu_out) {
  if (or_nparams(m) < 0 || nx <= 0 || ny <= 0 || !th || !range4 || !mu_out) return -1;
  for (int64_t i = 0; i < nx * ny; ++i) mu_out[i] = eval_mu(m, th, nx, ny, range4, NULL, i, NULL);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Objective term l(n, mu) and dl/dmu.                                     */
/* Returns 0 for a regular term, 1 for a domain error (l = +inf, ubar = 0),*/
/* 2 for a skipped bin (l = 0, ubar = 0).                                  */
/* ---------------------------------------------------------------------- */
static int objective_term(int obj, double n, double mu, double* l, double* ubar) {
  switch (obj) {
    case OR_NEYMAN:
      if (!(n > 0.0)) {
        *l = 0.0;
        *ubar = 0.0;
        return 2;
      }
      *l = (n - mu) * (n - mu) / n;
      *ubar = 2.0 * (mu - n) / n;
      return 0;
    case OR_PEARSON:
      if (!(mu > 0.0)) break;
      *l = (n - mu) * (n - mu) / mu;
      *ubar = 1.0 - (n * n) / (mu * mu);
      return 0;
    case OR_POISSON:
      if (n > 0.0) {
        if (!(mu > 0.0)) break;
        *l = mu - n + n * log(n / mu);
        *ubar = 1.0 - n / mu;
        return 0;
      }
      if (mu < 0.0) break;
      *l = mu;
      *ubar = 1.0;
      return 0;
    default:
      break;
  }
  *l = INFINITY;
  *ubar = 0.0;
  return 1;
}

/* ---------------------------------------------------------------------- */
/* NLL and gradient                                                        */
/* ---------------------------------------------------------------------- */
typedef struct {
  const or_model* m;
  int obj;
  const double* counts;
  const double* weights;
  int64_t nx, ny;
  const double* range;
  const double* edges;
  const double* th;
  int P;
  int64_t begin, end;
  int want_grad;
  double* ell_out;
  /* results */
  nsum nll, nll_abs;
  nsum grad[OR_MAXP], grad_abs[OR_MAXP];
  int status;
} chunk_job;

static void run_chunk(chunk_job* j) {
  double dmu[OR_MAXP];
  memset(&j->nll, 0, sizeof(j->nll));
  memset(&j->nll_abs, 0, sizeof(j->nll_abs));
  memset(j->grad, 0, sizeof(j->grad));
  memset(j->grad_abs, 0, sizeof(j->grad_abs));
  j->status = 0;
  for (int64_t i = j->begin; i < j->end; ++i) {
    double n = j->counts[i];
    double w = j->weights ? j->weights[i] : 1.0;
    double mu = eval_mu(j->m, j->th, j->nx, j->ny, j->range, j->edges, i,
                        j->want_grad ? dmu : NULL);
    double l, ubar;
    int rc = objective_term(j->obj, n, mu, &l, &ubar);
    if (rc == 1) j->status |= OR_ST_DOMAIN;
    if (j->ell_out) j->ell_out[i] = l;
    nsum_add(&j->nll, w * l);
    nsum_add(&j->nll_abs, fabs(w * l));
    if (j->want_grad && rc == 0) {
      for (int k = 0; k < j->P; ++k) {
        double g = w * ubar * dmu[k];
        nsum_add(&j->grad[k], g);
        nsum_add(&j->grad_abs[k], fabs(g));
      }
    }
  }
}

static void* chunk_thread(void* arg) {
  run_chunk((chunk_job*)arg);
  return NULL;
}

static int theta_finite(const double* th, int P) {
  for (int k = 0; k < P; ++k)
    if (!isfinite(th[k])) return 0;
  return 1;
}

/* Evaluates L(theta) and, when grad_out != NULL, dL/dtheta.  scale_out
 * (nullable, P+1 values) receives S_0 then S_1..S_P; ell_out (nullable,
 * nx*ny values) receives the unweighted per-bin terms l_i.  nthreads > 1
 * splits the bins into nthreads contiguous chunks, each summed as above,
 * and combines the chunk sums in chunk order.                            */
static int nll_grad_impl(const or_model* m, int obj, const double* counts, const double* weights,
                         int64_t nx, int64_t ny, const double* range4, const double* edges,
                         const double* theta, double* nll_out, double* grad_out,
                         double* scale_out, double* ell_out, int32_t* status_out, int nthreads) {
  int P = or_nparams(m);
  if (P < 0 || P > OR_MAXP) return -2;
  if (!counts || !range4 || !theta || !nll_out || nx <= 0 || ny <= 0) return -1;
  if (m->kind != OR_GAUSS2D && ny != 1) return -1;
  if (obj < OR_NEYMAN || obj > OR_POISSON) return -2;
  if (nthreads < 1) nthreads = 1;
  int64_t nb = nx * ny;
  if ((int64_t)nthreads > nb) nthreads = (int)nb;

  chunk_job* jobs = (chunk_job*)calloc((size_t)nthreads, sizeof(chunk_job));
  pthread_t* tids = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !tids) {
    free(jobs);
    free(tids);
    return -4;
  }
  for (int t = 0; t < nthreads; ++t) {
    chunk_job* j = &jobs[t];
    j->m = m;
    j->obj = obj;
    j->counts = counts;
    j->weights = weights;
    j->nx = nx;
    j->ny = ny;
    j->range = range4;
    j->edges = edges;
    j->th = theta;
    j->P = P;
    j->begin = nb * t / nthreads;
    j->end = nb * (t + 1) / nthreads;
    j->want_grad = (grad_out != NULL) || (scale_out != NULL);
    j->ell_out = ell_out;
  }
  if (nthreads == 1) {
    run_chunk(&jobs[0]);
  } else {
    for (int t = 0; t < nthreads; ++t) pthread_create(&tids[t], NULL, chunk_thread, &jobs[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(tids[t], NULL);
  }
  nsum nll = {0, 0}, nll_abs = {0, 0};
  nsum grad[OR_MAXP], grad_abs[OR_MAXP];
  memset(grad, 0, sizeof(grad));
  memset(grad_abs, 0, sizeof(grad_abs));
  int status = 0;
  for (int t = 0; t < nthreads; ++t) {
    chunk_job* j = &jobs[t];
    status |= j->status;
    nsum_add(&nll, j->nll.s);
    nsum_add(&nll, j->nll.c);
    nsum_add(&nll_abs, j->nll_abs.s);
    nsum_add(&nll_abs, j->nll_abs.c);
    for (int k = 0; k < P; ++k) {
      nsum_add(&grad[k], j->grad[k].s);
      nsum_add(&grad[k], j->grad[k].c);
      nsum_add(&grad_abs[k], j->grad_abs[k].s);
      nsum_add(&grad_abs[k], j->grad_abs[k].c);
    }
  }
  free(jobs);
  free(tids);
  if (!theta_finite(theta, P)) status |= OR_ST_NONFINITE;
  *nll_out = nsum_value(&nll);
  if (grad_out)
    for (int k = 0; k < P; ++k) grad_out[k] = (status & OR_ST_DOMAIN) ? NAN : nsum_value(&grad[k]);
  if (scale_out) {
    scale_out[0] = nsum_value(&nll_abs);
    for (int k = 0; k < P; ++k) scale_out[1 + k] = nsum_value(&grad_abs[k]);
  }
  if (status_out) *status_out = status;
  return 0;
}

int or_nll_grad_mt(const or_model* m, int obj, const double* counts, const double* weights,
                   int64_t nx, int64_t ny, const double* range4, const double* theta,
                   double* nll_out, double* grad_out, double* scale_out, double* ell_out,
                   int32_t* status_out, int nthreads) {
  return nll_grad_impl(m, obj, counts, weights, nx, ny, range4, NULL, theta, nll_out, grad_out,
                       scale_out, ell_out, status_out, nthreads);
}

/* As or_nll_grad_mt for a 1D histogram with bins of any widths: bin i spans
 * [edges[i], edges[i+1]] (nx + 1 ascending edges); the model is taken at
 * the midpoint, or averaged over the bin for bin-average models.          */
int or_nll_grad_edges(const or_model* m, int obj, const double* counts, const double* weights,
                      int64_t nx, const double* edges, const double* theta, double* nll_out,
                      double* grad_out, double* scale_out, double* ell_out, int32_t* status_out,
                      int nthreads) {
  if (!edges || nx <= 0 || m->kind == OR_GAUSS2D) return -1;
  for (int64_t i = 0; i < nx; ++i)
    if (!(edges[i + 1] > edges[i])) return -1;
  double r[4] = {edges[0], edges[nx], 0.0, 1.0};
  return nll_grad_impl(m, obj, counts, weights, nx, 1, r, edges, theta, nll_out, grad_out,
                       scale_out, ell_out, status_out, nthreads);
}

int or_nll_grad(const or_model* m, int obj, const double* counts, const double* weights,
                int64_t nx, int64_t ny, const double* range4, const double* theta,
                double* nll_out, double* grad_out, double* scale_out, double* ell_out,
                int32_t* status_out) {
  return or_nll_grad_mt(m, obj, counts, weights, nx, ny, range4, theta, nll_out, grad_out,
                        scale_out, ell_out, status_out, 1);
}

/* ---------------------------------------------------------------------- */
/* Extended unbinned NLL (per-event evaluation of the same 1D intensity)  */
/* ---------------------------------------------------------------------- */
/* For events x_e (weights w_e, default 1) and the 1D Gauss + polynomial
 * model read as an intensity lambda(x; theta) (events per unit x):
 *   L(theta) = Lambda(theta) - sum_e w_e ln lambda(x_e),
 *   Lambda   = integral of lambda over [lo, hi],
 * the extended likelihood of a Poisson process, whose per-event terms are
 * the binned objective's bins shrunk to single events.  Lambda in closed
 * form, per Gaussian with z_b = (b - m)/s, e_b = exp(-z_b^2/2):
 *   Lambda_g      = A s sqrt(pi/2) [erf(z_hi/sqrt 2) - erf(z_lo/sqrt 2)]
 *   dLambda_g/dA  = Lambda_g / A  (written as s sqrt(pi/2) [erf difference])
 *   dLambda_g/dm  = A (e_lo - e_hi)
 *   dLambda_g/ds  = Lambda_g / s + A (z_lo e_lo - z_hi e_hi)
 * and for the polynomial in t = (x - t_shift)/t_scale
 *   dLambda/dc_j  = t_scale (t_hi^(j+1) - t_lo^(j+1)) / (j + 1).
 * The event terms' gradient is -sum_e w_e (dlambda/dtheta)(x_e) / lambda(x_e)
 * with the closed-form partials of model1d.  Events outside [lo, hi] are
 * skipped; lambda <= 0 at an event inside is a domain error (L = +inf,
 * status bit 0).  Sums are Neumaier-compensated in event order; scale_out
 * (P+1 values, or NULL) receives |Lambda| + sum|w ln lambda| and, per
 * parameter, |dLambda/dtheta_k| + sum|w dlambda_k / lambda|.  Kinds 1 and 2
 * (the exponential's integral is (hi - lo) E_c S(b1 d) with E_c at the
 * range's midpoint t_c and d its half-width in t; see sinhc).
 * Returns 0, -1 on bad arguments, -2 for an unsupported model.           */
int or_unbinned(const or_model* m, const double* x, const double* weights, int64_t n, double lo,
                double hi, const double* theta, double* nll_out, double* grad_out,
                double* scale_out, int32_t* status_out) {
  int P = or_nparams(m);
  if (P < 0 || P > OR_MAXP || m->kind == OR_GAUSS2D) return -2;
  if ((n > 0 && !x) || !theta || !nll_out || !(hi > lo)) return -1;
  int32_t status = theta_finite(theta, P) ? 0 : OR_ST_NONFINITE;
  /* Lambda and its gradient */
  double lam_tot = 0.0, dlam[OR_MAXP];
  int k = 0;
  const double rt = sqrt(0.5 * 3.14159265358979323846), r2 = sqrt(2.0);
  for (int g = 0; g < m->n_gauss; ++g, k += 3) {
    double A = theta[k], mean = theta[k + 1], s = theta[k + 2];
    double zl = (lo - mean) / s, zh = (hi - mean) / s;
    double el = exp(-0.5 * zl * zl), eh = exp(-0.5 * zh * zh);
    double ia = s * rt * (erf(zh / r2) - erf(zl / r2));
    double lg = A * ia;
    lam_tot += lg;
    dlam[k] = ia;
    dlam[k + 1] = A * (el - eh);
    dlam[k + 2] = lg / s + A * (zl * el - zh * eh);
  }
  double tl = (lo - m->t_shift) / m->t_scale, th = (hi - m->t_shift) / m->t_scale;
  if (m->kind == OR_GAUSS_EXP) {
    /* integral of exp(b0 + b1 t) over the range: (hi - lo) E_c S(b1 d) */
    double tc = 0.5 * (tl + th), d = 0.5 * (th - tl), S, dS;
    double Ec = exp(theta[k] + theta[k + 1] * tc);
    sinhc(theta[k + 1] * d, &S, &dS);
    lam_tot += (hi - lo) * Ec * S;
    dlam[k] = (hi - lo) * Ec * S;
    dlam[k + 1] = (hi - lo) * Ec * (tc * S + d * dS);
  }
  for (int j = 0; m->kind == OR_GAUSS_POLY && j <= m->poly_degree; ++j) {
    double ij = m->t_scale * (pow(th, j + 1) - pow(tl, j + 1)) / (j + 1);
    lam_tot += theta[k + j] * ij;
    dlam[k + j] = ij;
  }
  /* event terms */
  nsum sl = {0.0, 0.0}, sg[OR_MAXP];
  double al = 0.0, ag[OR_MAXP];
  for (int a = 0; a < P; ++a) {
    sg[a].s = sg[a].c = 0.0;
    ag[a] = 0.0;
  }
  double dmu[OR_MAXP];
  for (int64_t e = 0; e < n; ++e) {
    if (!(x[e] >= lo && x[e] <= hi)) continue;
    double w = weights ? weights[e] : 1.0;
    double lam = model1d(m, theta, x[e], dmu);
    if (!(lam > 0.0)) {
      status |= OR_ST_DOMAIN;
      continue;
    }
    double t = w * log(lam);
    nsum_add(&sl, t);
    al += fabs(t);
    for (int a = 0; a < P; ++a) {
      double v = w * dmu[a] / lam;
      nsum_add(&sg[a], v);
      ag[a] += fabs(v);
    }
  }
  double nan = NAN;
  if (status & OR_ST_NONFINITE) {
    *nll_out = nan;
    if (grad_out)
      for (int a = 0; a < P; ++a) grad_out[a] = nan;
  } else if (status & OR_ST_DOMAIN) {
    *nll_out = INFINITY;
    if (grad_out)
      for (int a = 0; a < P; ++a) grad_out[a] = nan;
  } else {
    *nll_out = lam_tot - nsum_value(&sl);
    if (grad_out)
      for (int a = 0; a < P; ++a) grad_out[a] = dlam[a] - nsum_value(&sg[a]);
  }
  if (scale_out) {
    scale_out[0] = fabs(lam_tot) + al;
    for (int a = 0; a < P; ++a) scale_out[1 + a] = fabs(dlam[a]) + ag[a];
  }
  if (status_out) *status_out = status;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* BFGS fitter                                                             */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t max_iter;
  int32_t ls_max;
  int32_t fixed_iters; /* nonzero: ignore the EDM test, run max_iter steps */
  uint32_t free_mask;  /* bit k set: theta_k is free; 0 means all free   */
  double edm_tol;
  int32_t hessian_init; /* 0: H = I; 1: H = inverse expected Hessian at theta0 */
  int32_t reserved;
} or_fit_opts;

/* Expected Hessian (Fisher information) of L = sum_i w_i l_i:
 *   F = sum_i w_i c_i (dmu_i/dtheta)(dmu_i/dtheta)^T
 * with c_i = d^2 l / d mu^2 at n_i = mu_i: 1/mu_i (Poisson), 2/n_i for
 * n_i > 0 (Neyman; empty bins are skipped), 2/mu_i (Pearson).  Where the
 * counts equal the model this is the exact Hessian, because the second
 * derivatives of mu are multiplied by dl/dmu = 0.  Bins whose c_i is not a
 * finite positive number (mu <= 0) contribute nothing.  F_out is row-major
 * P x P, each entry a Neumaier sum in bin order.  Returns 0, or -1/-2 on
 * bad arguments.                                                         */
int or_fisher(const or_model* m, int obj, const double* counts, const double* weights, int64_t nx,
              int64_t ny, const double* range4, const double* theta, double* F_out) {
  int P = or_nparams(m);
  if (P < 0 || P > OR_MAXP) return -2;
  if (!counts || !range4 || !theta || !F_out || nx <= 0 || ny <= 0) return -1;
  nsum* acc = (nsum*)calloc((size_t)P * (size_t)P, sizeof(nsum));
  if (!acc) return -1;
  double dmu[OR_MAXP];
  for (int64_t i = 0; i < nx * ny; ++i) {
    double n = counts[i];
    double w = weights ? weights[i] : 1.0;
    double mu = eval_mu(m, theta, nx, ny, range4, NULL, i, dmu);
    double c;
    if (obj == OR_POISSON) c = 1.0 / mu;
    else if (obj == OR_PEARSON) c = 2.0 / mu;
    else c = (n > 0.0) ? 2.0 / n : 0.0;
    if (!(c > 0.0) || !isfinite(c)) continue;
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b) nsum_add(&acc[a * P + b], w * c * dmu[a] * dmu[b]);
  }
  for (int a = 0; a < P * P; ++a) F_out[a] = nsum_value(&acc[a]);
  free(acc);
  return 0;
}

/* Inverse of the symmetric n x n matrix A (row-major) by Cholesky,
 * A = L L^T, then inv(A) = inv(L)^T inv(L).  Fails (returns 0) when a pivot
 * is not above 1e-12 times the largest diagonal entry or anything is not
 * finite; returns 1 with the inverse in Ainv otherwise.                   */
static int spd_inverse(const double* A, int n, double* Ainv) {
  double L[OR_MAXP * OR_MAXP] = {0}, Li[OR_MAXP * OR_MAXP] = {0};
  double dmax = 0.0;
  for (int a = 0; a < n; ++a) dmax = fmax(dmax, A[a * n + a]);
  if (!(dmax > 0.0) || !isfinite(dmax)) return 0;
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 1e-12 * dmax) || !isfinite(d)) return 0;
    L[j * n + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  /* inv(L) by forward substitution, column by column */
  for (int c = 0; c < n; ++c) {
    for (int i = c; i < n; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= L[i * n + k] * Li[k * n + c];
      Li[i * n + c] = v / L[i * n + i];
    }
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double v = 0.0;
      for (int k = (a > b ? a : b); k < n; ++k) v += Li[k * n + a] * Li[k * n + b];
      Ainv[a * n + b] = v;
    }
  for (int a = 0; a < n * n; ++a)
    if (!isfinite(Ainv[a])) return 0;
  return 1;
}

enum { OR_FIT_CONVERGED = 0, OR_FIT_MAXITER = 1, OR_FIT_LSFAIL = 2, OR_FIT_NONFINITE = 3,
       OR_FIT_DOMAIN = 4 };

/* Scale of each parameter for the fitter's internal coordinates
 * u_k = (theta_k - theta0_k) / sigma_k, chosen by the parameter's kind.  */
static void param_scales(const or_model* m, const double* th0, const double* range4, double* sig) {
  double rx = range4[1] - range4[0];
  if (m->kind == OR_GAUSS2D) {
    double ry = range4[3] - range4[2];
    sig[0] = fmax(fabs(th0[0]), 1.0);
    sig[1] = rx / 100.0;
    sig[2] = ry / 100.0;
    sig[3] = fabs(th0[3]) > 0 ? fabs(th0[3]) : rx / 100.0;
    sig[4] = fabs(th0[4]) > 0 ? fabs(th0[4]) : ry / 100.0;
    sig[5] = 0.1;
    sig[6] = fmax(fabs(th0[6]), 1.0);
    return;
  }
  int k = 0;
  for (int g = 0; g < m->n_gauss; ++g, k += 3) {
    sig[k] = fmax(fabs(th0[k]), 1.0);
    sig[k + 1] = rx / 100.0;
    sig[k + 2] = fabs(th0[k + 2]) > 0 ? fabs(th0[k + 2]) : rx / 100.0;
  }
  int nb = (m->kind == OR_GAUSS_POLY) ? m->poly_degree + 1 : 2;
  for (int j = 0; j < nb; ++j) sig[k + j] = fmax(fabs(th0[k + j]), 1.0);
}

/* Puts a fitted parameter vector in canonical form: |s| for every width,
 * Gaussians ordered by mean (stable), and for the 2D model the sign of rho
 * flipped when exactly one width was negative.                           */
static void canonicalise(const or_model* m, double* th) {
  if (m->kind == OR_GAUSS2D) {
    int flip = (th[3] < 0) != (th[4] < 0);
    th[3] = fabs(th[3]);
    th[4] = fabs(th[4]);
    if (flip) th[5] = -th[5];
    return;
  }
  for (int g = 0; g < m->n_gauss; ++g) th[3 * g + 2] = fabs(th[3 * g + 2]);
  for (int a = 1; a < m->n_gauss; ++a) {
    for (int b = a; b > 0 && th[3 * b + 1] < th[3 * (b - 1) + 1]; --b) {
      for (int q = 0; q < 3; ++q) {
        double tmp = th[3 * b + q];
        th[3 * b + q] = th[3 * (b - 1) + q];
        th[3 * (b - 1) + q] = tmp;
      }
    }
  }
}

typedef struct {
  const or_model* m;
  int obj;
  const double* counts;
  const double* weights;
  int64_t nx, ny;
  const double* range;
  const double* th0;
  const double* sig;
  const int* fidx;
  int nf, P;
  int nthreads;
  int nevals;
} fit_problem;

/* f(u) and its gradient with respect to the free internal coordinates.   */
static double fit_eval(fit_problem* fp, const double* u, double* gu, double* th) {
  double grad[OR_MAXP];
  memcpy(th, fp->th0, sizeof(double) * (size_t)fp->P);
  for (int a = 0; a < fp->nf; ++a) th[fp->fidx[a]] = fp->th0[fp->fidx[a]] + fp->sig[fp->fidx[a]] * u[a];
  double nll;
  int32_t st = 0;
  or_nll_grad_mt(fp->m, fp->obj, fp->counts, fp->weights, fp->nx, fp->ny, fp->range, th, &nll,
                 grad, NULL, NULL, &st, fp->nthreads);
  fp->nevals++;
  for (int a = 0; a < fp->nf; ++a) gu[a] = fp->sig[fp->fidx[a]] * grad[fp->fidx[a]];
  return nll;
}

int or_fit_mt(const or_model* m, int obj, const double* counts, const double* weights, int64_t nx,
              int64_t ny, const double* range4, const double* theta0, const or_fit_opts* opts,
              double* theta_out, double* nll_out, int32_t* status_out, int32_t* iters_out,
              int32_t* nevals_out, int nthreads) {
  int P = or_nparams(m);
  if (P < 0 || P > OR_MAXP) return -2;
  if (!counts || !range4 || !theta0 || !opts || !theta_out || !nll_out) return -1;
  const double c1 = 1e-4;
  double sig[OR_MAXP];
  int fidx[OR_MAXP];
  int nf = 0;
  param_scales(m, theta0, range4, sig);
  for (int k = 0; k < P; ++k)
    if (opts->free_mask == 0 || (opts->free_mask >> k) & 1u) fidx[nf++] = k;

  fit_problem fp = {m, obj, counts, weights, nx, ny, range4, theta0, sig, fidx, nf, P, nthreads, 0};
  double u[OR_MAXP] = {0}, g[OR_MAXP], un[OR_MAXP], gn[OR_MAXP], p[OR_MAXP], th[OR_MAXP];
  double H[OR_MAXP * OR_MAXP];
  double Hy[OR_MAXP];
  for (int a = 0; a < nf * nf; ++a) H[a] = 0.0;
  for (int a = 0; a < nf; ++a) H[a * nf + a] = 1.0;
  int first_update = 1;
  if (opts->hessian_init == 1 && nf > 0) {
    /* H = inverse of the expected Hessian at theta0 in the internal
     * coordinates (F_u = diag(sigma) F diag(sigma) over the free
     * parameters); identity when F_u is not safely positive definite.   */
    double F[OR_MAXP * OR_MAXP], Fu[OR_MAXP * OR_MAXP], Hi[OR_MAXP * OR_MAXP];
    if (or_fisher(m, obj, counts, weights, nx, ny, range4, theta0, F) == 0) {
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b)
          Fu[a * nf + b] = sig[fidx[a]] * sig[fidx[b]] * F[fidx[a] * P + fidx[b]];
      if (spd_inverse(Fu, nf, Hi)) {
        for (int a = 0; a < nf * nf; ++a) H[a] = Hi[a];
        first_update = 0;
      }
    }
  }

  double f = fit_eval(&fp, u, g, th);
  int status = OR_FIT_MAXITER;
  int it = 0;
  if (!isfinite(f)) {
    status = (f == INFINITY) ? OR_FIT_DOMAIN : OR_FIT_NONFINITE;
  } else {
    for (; it < opts->max_iter;) {
      /* EDM = g^T H g / 2 */
      double edm = 0.0;
      for (int a = 0; a < nf; ++a) {
        double hg = 0.0;
        for (int b = 0; b < nf; ++b) hg += H[a * nf + b] * g[b];
        p[a] = -hg;
        edm += g[a] * hg;
      }
      edm *= 0.5;
      /* An EDM below a few ulps of |f| cannot be verified by comparing f
       * values, so it counts as converged whatever edm_tol asks for.      */
      double edm_goal = fmax(opts->edm_tol, 4.0 * DBL_EPSILON * fabs(f));
      if (!opts->fixed_iters && edm < edm_goal) {
        status = OR_FIT_CONVERGED;
        break;
      }
      double slope = 0.0;
      for (int a = 0; a < nf; ++a) slope += g[a] * p[a];
      if (!(slope < 0.0)) { /* H lost positive definiteness: restart from I */
        for (int a = 0; a < nf * nf; ++a) H[a] = 0.0;
        for (int a = 0; a < nf; ++a) H[a * nf + a] = 1.0;
        first_update = 1;
        slope = 0.0;
        for (int a = 0; a < nf; ++a) {
          p[a] = -g[a];
          slope -= g[a] * g[a];
        }
      }
      /* backtracking Armijo: halve alpha until f(u + alpha p) <= f + c1 alpha slope */
      double alpha = 1.0, fn = 0.0;
      int accepted = 0;
      for (int ls = 0; ls < opts->ls_max; ++ls) {
        for (int a = 0; a < nf; ++a) un[a] = u[a] + alpha * p[a];
        fn = fit_eval(&fp, un, gn, th);
        if (isfinite(fn) && fn <= f + c1 * alpha * slope) {
          accepted = 1;
          break;
        }
        alpha *= 0.5;
      }
      if (!accepted) {
        status = (edm < edm_goal) ? OR_FIT_CONVERGED : OR_FIT_LSFAIL;
        break;
      }
      ++it;
      /* s = alpha p, y = g_new - g; BFGS inverse update when s^T y is safely positive */
      double s[OR_MAXP], y[OR_MAXP], sy = 0.0, yy = 0.0, ss = 0.0;
      for (int a = 0; a < nf; ++a) {
        s[a] = un[a] - u[a];
        y[a] = gn[a] - g[a];
        sy += s[a] * y[a];
        yy += y[a] * y[a];
        ss += s[a] * s[a];
      }
      if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
        if (first_update) {
          double gam = sy / yy;
          for (int a = 0; a < nf * nf; ++a) H[a] *= gam;
          first_update = 0;
        }
        double rho = 1.0 / sy, yHy = 0.0;
        for (int a = 0; a < nf; ++a) {
          double acc = 0.0;
          for (int b = 0; b < nf; ++b) acc += H[a * nf + b] * y[b];
          Hy[a] = acc;
          yHy += y[a] * acc;
        }
        for (int a = 0; a < nf; ++a)
          for (int b = 0; b < nf; ++b)
            H[a * nf + b] += -rho * (Hy[a] * s[b] + s[a] * Hy[b]) + (rho * rho * yHy + rho) * s[a] * s[b];
      }
      for (int a = 0; a < nf; ++a) {
        u[a] = un[a];
        g[a] = gn[a];
      }
      f = fn;
    }
  }
  memcpy(theta_out, theta0, sizeof(double) * (size_t)P);
  for (int a = 0; a < nf; ++a) theta_out[fidx[a]] = theta0[fidx[a]] + sig[fidx[a]] * u[a];
  canonicalise(m, theta_out);
  *nll_out = f;
  if (status_out) *status_out = status;
  if (iters_out) *iters_out = it;
  if (nevals_out) *nevals_out = fp.nevals;
  return 0;
}

int or_fit(const or_model* m, int obj, const double* counts, const double* weights, int64_t nx,
           int64_t ny, const double* range4, const double* theta0, const or_fit_opts* opts,
           double* theta_out, double* nll_out, int32_t* status_out, int32_t* iters_out,
           int32_t* nevals_out) {
  return or_fit_mt(m, obj, counts, weights, nx, ny, range4, theta0, opts, theta_out, nll_out,
                   status_out, iters_out, nevals_out, 1);
}

/* Independent fits of B histograms laid end to end (offsets[b]..offsets[b+1]
 * in counts, ranges[2b], ranges[2b+1]), spread over nthreads host threads
 * by histogram; each fit is single-threaded.                              */
typedef struct {
  const or_model* m;
  int obj;
  const double* counts;
  const int64_t* offsets;
  const double* ranges;
  const double* theta0;
  const or_fit_opts* opts;
  double* theta_out;
  double* nll_out;
  int32_t* status;
  int32_t* iters;
  int32_t* nevals;
  int P;
  int B;
  int tid, nthreads;
} batch_job;

static void* batch_thread(void* arg) {
  batch_job* j = (batch_job*)arg;
  for (int b = j->tid; b < j->B; b += j->nthreads) {
    double r4[4] = {j->ranges[2 * b], j->ranges[2 * b + 1], 0.0, 1.0};
    int64_t nb = j->offsets[b + 1] - j->offsets[b];
    or_fit(j->m, j->obj, j->counts + j->offsets[b], NULL, nb, 1, r4, j->theta0 + (size_t)b * j->P,
           j->opts, j->theta_out + (size_t)b * j->P, j->nll_out + b, j->status + b, j->iters + b,
           j->nevals + b);
  }
  return NULL;
}

int or_fit_many(const or_model* m, int obj, int32_t B, const double* counts, const int64_t* offsets,
                const double* ranges, const double* theta0, const or_fit_opts* opts,
                double* theta_out, double* nll_out, int32_t* status, int32_t* iters,
                int32_t* nevals, int nthreads) {
  int P = or_nparams(m);
  if (P < 0 || m->kind == OR_GAUSS2D) return -2;
  if (B < 0 || !counts || !offsets || !ranges || !theta0 || !opts || !theta_out || !nll_out ||
      !status || !iters || !nevals)
    return -1;
  if (nthreads < 1) nthreads = 1;
  batch_job* jobs = (batch_job*)calloc((size_t)nthreads, sizeof(batch_job));
  pthread_t* tids = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !tids) {
    free(jobs);
    free(tids);
    return -4;
  }
  for (int t = 0; t < nthreads; ++t) {
    batch_job j = {m, obj, counts, offsets, ranges, theta0, opts, theta_out, nll_out,
                   status, iters, nevals, P, B, t, nthreads};
    jobs[t] = j;
    pthread_create(&tids[t], NULL, batch_thread, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(tids[t], NULL);
  free(jobs);
  free(tids);
  return 0;
}
