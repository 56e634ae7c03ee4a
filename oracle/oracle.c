/*
 * oracle.c -- plain, slow, FP64 CPU reference for the MGRIT + p-multigrid solver of
 * Tielen, Moeller and Vuik, "Combining p-multigrid and multigrid reduced in time methods
 * to obtain a scalable solver for Isogeometric Analysis" (arXiv 2107.05337).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the GPU library and never calls it.
 *
 * Every routine follows the paper's definitions in the paper's order, without blocking or
 * fusion:
 *   - open uniform knot vectors and the Cox-de Boor recursion (Sec. 2, Cox-de Boor formula),
 *   - the tensor-product spline space on a single patch F : (0,1)^2 -> Omega (Sec. 2),
 *   - mass and stiffness matrices by an element loop with Gauss quadrature (Sec. 2, eq:los),
 *   - the linear system of each implicit Euler step, theta = 1 (Sec. 2, eq:los; Sec. 4),
 *   - ILUT (Saad's dual-threshold incomplete LU; the smoother named in Sec. 4),
 *   - the p-multigrid V-cycle, steps 1-5, with L2-projection transfers built from the
 *     row-sum-lumped mass matrices (Sec. 4, eq:prolongation, eq:PM),
 *   - an exact (direct) solve at p = 1 by banded Cholesky,
 *   - sequential implicit Euler with direct solves (the block forward solve of eq:mgrit),
 *   - two-level and multilevel MGRIT with FCF-relaxation, injection and ideal interpolation
 *     (Sec. 3, eq:mgrit_coarse and the MGRIT recursion).
 * Readings where the paper is silent are listed in the repository's design notes and are
 * restated next to the code that takes them.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* small utilities                                                     */
/* ------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s ? s : 1);
  if (!p) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  return p;
}

/* compressed sparse row matrix, sorted column indices */
typedef struct {
  int nr, nc, nnz;
  int *rp, *ci;
  double *v;
} ocsr;

static void csr_free(ocsr *a) {
  free(a->rp);
  free(a->ci);
  free(a->v);
  memset(a, 0, sizeof(*a));
}

/* y = A x */
static void csr_mv(const ocsr *a, const double *x, double *y) {
  for (int i = 0; i < a->nr; ++i) {
    double s = 0.0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) s += a->v[k] * x[a->ci[k]];
    y[i] = s;
  }
}

/* y = A^T x */
static void csr_mtv(const ocsr *a, const double *x, double *y) {
  for (int j = 0; j < a->nc; ++j) y[j] = 0.0;
  for (int i = 0; i < a->nr; ++i)
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) y[a->ci[k]] += a->v[k] * x[i];
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

/* ------------------------------------------------------------------ */
/* B-splines (Sec. 2)                                                  */
/* ------------------------------------------------------------------ */

/* Open uniform knot vector on [0,1] with n elements of width h = 1/n; the first and last
 * knots are repeated p+1 times (Sec. 2).  Length n + 2p + 1, giving N = n + p functions. */
ORC_API void orc_knots(int p, int n, double *xi) {
  int k = 0;
  for (int i = 0; i < p; ++i) xi[k++] = 0.0;
  for (int i = 0; i <= n; ++i) xi[k++] = (double)i / (double)n;
  for (int i = 0; i < p; ++i) xi[k++] = 1.0;
}

/* Cox-de Boor recursion (Sec. 2): phi_{i,0} = 1 on [xi_i, xi_{i+1}), and
 * phi_{i,p} = (x - xi_i)/(xi_{i+p} - xi_i) phi_{i,p-1} + (xi_{i+p+1} - x)/(xi_{i+p+1} - xi_{i+1}) phi_{i+1,p-1},
 * with the usual convention 0/0 := 0.  Index i is 0-based.  At the right end of the knot
 * vector the last non-empty span is taken closed, so that the basis stays interpolatory
 * there (the property stated in Sec. 2). */
ORC_API double orc_bspline(const double *xi, int nk, int i, int p, double x) {
  if (p == 0) {
    double a = xi[i], b = xi[i + 1];
    if (a <= x && x < b) return 1.0;
    if (x == xi[nk - 1] && a < b && b == xi[nk - 1]) return 1.0;
    return 0.0;
  }
  double r = 0.0;
  double d1 = xi[i + p] - xi[i];
  double d2 = xi[i + p + 1] - xi[i + 1];
  if (d1 > 0.0) r += (x - xi[i]) / d1 * orc_bspline(xi, nk, i, p - 1, x);
  if (d2 > 0.0) r += (xi[i + p + 1] - x) / d2 * orc_bspline(xi, nk, i + 1, p - 1, x);
  return r;
}

/* Derivative of phi_{i,p}: the textbook formula (de Boor)
 * p/(xi_{i+p} - xi_i) phi_{i,p-1} - p/(xi_{i+p+1} - xi_{i+1}) phi_{i+1,p-1}. */
ORC_API double orc_bspline_deriv(const double *xi, int nk, int i, int p, double x) {
  if (p == 0) return 0.0;
  double r = 0.0;
  double d1 = xi[i + p] - xi[i];
  double d2 = xi[i + p + 1] - xi[i + 1];
  if (d1 > 0.0) r += (double)p / d1 * orc_bspline(xi, nk, i, p - 1, x);
  if (d2 > 0.0) r -= (double)p / d2 * orc_bspline(xi, nk, i + 1, p - 1, x);
  return r;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre quadrature on [0,1] (textbook: Newton on P_q)        */
/* ------------------------------------------------------------------ */

ORC_API void orc_gauss(int q, double *x01, double *w01) {
  for (int i = 0; i < q; ++i) {
    double z = cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
    }
    double w = 2.0 / ((1.0 - z * z) * dp * dp);
    /* map from [-1,1] to [0,1]; nodes in increasing order */
    x01[q - 1 - i] = 0.5 * (z + 1.0);
    w01[q - 1 - i] = 0.5 * w;
  }
}

/* ------------------------------------------------------------------ */
/* Geometry F : (0,1)^2 -> Omega (Sec. 2)                              */
/* ------------------------------------------------------------------ */

/* domain 0: unit square, F = identity.
 * domain 1: quarter annulus with radii 1 and 2, written as a NURBS surface of degree
 * (1, 2): radial direction xi_1 linear between r = 1 and r = 2, angular direction xi_2 the
 * exact rational quadratic quarter circle with control points (1,0), (1,1), (0,1) and
 * weights 1, sqrt(2)/2, 1.  The map is evaluated from the general NURBS formula
 * F = sum N_a N_b w_ab P_ab / sum N_a N_b w_ab with its quotient-rule derivatives. */
static void geom_eval(int domain, double s, double t, double *X, double J[2][2]) {
  if (domain == 0) {
    X[0] = s;
    X[1] = t;
    J[0][0] = 1.0;
    J[0][1] = 0.0;
    J[1][0] = 0.0;
    J[1][1] = 1.0;
    return;
  }
  static const double kr[4] = {0, 0, 1, 1};
  static const double kt[6] = {0, 0, 0, 1, 1, 1};
  const double w2 = sqrt(0.5);
  const double wt[3] = {1.0, w2, 1.0};
  const double cp[3][2] = {{1.0, 0.0}, {1.0, 1.0}, {0.0, 1.0}};
  double Sx = 0, Sy = 0, W = 0, Sx_s = 0, Sy_s = 0, W_s = 0, Sx_t = 0, Sy_t = 0, W_t = 0;
  for (int a = 0; a < 2; ++a) {
    double Na = orc_bspline(kr, 4, a, 1, s), dNa = orc_bspline_deriv(kr, 4, a, 1, s);
    double rad = 1.0 + (double)a;
    for (int b = 0; b < 3; ++b) {
      double Nb = orc_bspline(kt, 6, b, 2, t), dNb = orc_bspline_deriv(kt, 6, b, 2, t);
      double px = rad * cp[b][0], py = rad * cp[b][1], w = wt[b];
      W += Na * Nb * w;
      Sx += Na * Nb * w * px;
      Sy += Na * Nb * w * py;
      W_s += dNa * Nb * w;
      Sx_s += dNa * Nb * w * px;
      Sy_s += dNa * Nb * w * py;
      W_t += Na * dNb * w;
      Sx_t += Na * dNb * w * px;
      Sy_t += Na * dNb * w * py;
    }
  }
  X[0] = Sx / W;
  X[1] = Sy / W;
  J[0][0] = (Sx_s - X[0] * W_s) / W; /* dx/ds */
  J[0][1] = (Sx_t - X[0] * W_t) / W; /* dx/dt */
  J[1][0] = (Sy_s - X[1] * W_s) / W; /* dy/ds */
  J[1][1] = (Sy_t - X[1] * W_t) / W; /* dy/dt */
}

ORC_API void orc_geom(int domain, double s, double t, double *out6) {
  double X[2], J[2][2];
  geom_eval(domain, s, t, X, J);
  out6[0] = X[0];
  out6[1] = X[1];
  out6[2] = J[0][0];
  out6[3] = J[0][1];
  out6[4] = J[1][0];
  out6[5] = J[1][1];
}

/* ------------------------------------------------------------------ */
/* Assembly by an element loop (Sec. 2, eq:los and eq:PM)              */
/* ------------------------------------------------------------------ */

/* Sparse accumulation target: rows/cols of tensor-product functions whose supports overlap.
 * For bases of degrees pa (rows, Na functions per direction) and pb (cols, Nb per direction)
 * on the same n elements, row (ix,iy) couples to cols (jx,jy) with jx in [ix-pb, ix+pa]
 * clipped to [0, Nb).  The pattern is built first; entries are then added by binary search. */
static void pattern_tp(ocsr *a, int n, int pa, int pb) {
  int Na = n + pa, Nb = n + pb;
  a->nr = Na * Na;
  a->nc = Nb * Nb;
  a->rp = (int *)xcalloc((size_t)a->nr + 1, sizeof(int));
  /* 1D coupling range: function ix of degree pa lives on elements [ix-pa, ix]; function jx of
   * degree pb on [jx-pb, jx]; they overlap iff jx >= ix - pa and jx - pb <= ix */
  int cnt = 0;
  for (int iy = 0; iy < Na; ++iy)
    for (int ix = 0; ix < Na; ++ix) {
      int lox = ix - pa < 0 ? 0 : ix - pa, hix = ix + pb > Nb - 1 ? Nb - 1 : ix + pb;
      int loy = iy - pa < 0 ? 0 : iy - pa, hiy = iy + pb > Nb - 1 ? Nb - 1 : iy + pb;
      /* clip to functions that share at least one element */
      cnt += (hix - lox + 1) * (hiy - loy + 1);
    }
  a->nnz = cnt;
  a->ci = (int *)xcalloc((size_t)cnt, sizeof(int));
  a->v = (double *)xcalloc((size_t)cnt, sizeof(double));
  int k = 0;
  for (int iy = 0; iy < Na; ++iy)
    for (int ix = 0; ix < Na; ++ix) {
      int r = iy * Na + ix;
      a->rp[r] = k;
      int lox = ix - pa < 0 ? 0 : ix - pa, hix = ix + pb > Nb - 1 ? Nb - 1 : ix + pb;
      int loy = iy - pa < 0 ? 0 : iy - pa, hiy = iy + pb > Nb - 1 ? Nb - 1 : iy + pb;
      for (int jy = loy; jy <= hiy; ++jy)
        for (int jx = lox; jx <= hix; ++jx) a->ci[k++] = jy * Nb + jx;
    }
  a->rp[a->nr] = k;
}

static void csr_add(ocsr *a, int i, int j, double v) {
  int lo = a->rp[i], hi = a->rp[i + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (a->ci[mid] == j) {
      a->v[mid] += v;
      return;
    }
    if (a->ci[mid] < j)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  fprintf(stderr, "oracle: csr_add outside pattern (%d,%d)\n", i, j);
  abort();
}

/* Element-loop assembly on the full (pre-Dirichlet) spaces of degree pa (rows) and pb
 * (cols) over n x n elements with q Gauss points per direction:
 *   mass:      int Phi_i Phi_j dOmega                      (eq:los, eq:PM)
 *   stiffness: int grad Phi_i . grad Phi_j dOmega          (eq:los)
 * The integrand is evaluated at every 2D quadrature point with the geometry Jacobian of F
 * at that point; physical gradients are J^{-T} times parametric gradients. */
static void assemble_full(int domain, int n, int pa, int pb, int q, ocsr *mass, ocsr *stiff) {
  int nka = n + 2 * pa + 1, nkb = n + 2 * pb + 1;
  double *ka = (double *)xcalloc((size_t)nka, sizeof(double));
  double *kb = (double *)xcalloc((size_t)nkb, sizeof(double));
  orc_knots(pa, n, ka);
  orc_knots(pb, n, kb);
  double *gx = (double *)xcalloc((size_t)q, sizeof(double));
  double *gw = (double *)xcalloc((size_t)q, sizeof(double));
  orc_gauss(q, gx, gw);
  int Na = n + pa, Nb = n + pb, la = pa + 1, lb = pb + 1;
  if (mass) pattern_tp(mass, n, pa, pb);
  if (stiff) pattern_tp(stiff, n, pa, pb);
  double h = 1.0 / n;
  /* 1D values and derivatives of the functions living on an element, at its Gauss points */
  double *vax = (double *)xcalloc((size_t)q * la, sizeof(double)), *dax = (double *)xcalloc((size_t)q * la, sizeof(double));
  double *vay = (double *)xcalloc((size_t)q * la, sizeof(double)), *day = (double *)xcalloc((size_t)q * la, sizeof(double));
  double *vbx = (double *)xcalloc((size_t)q * lb, sizeof(double)), *dbx = (double *)xcalloc((size_t)q * lb, sizeof(double));
  double *vby = (double *)xcalloc((size_t)q * lb, sizeof(double)), *dby = (double *)xcalloc((size_t)q * lb, sizeof(double));
  double *em = (double *)xcalloc((size_t)la * la * lb * lb, sizeof(double));
  double *ek = (double *)xcalloc((size_t)la * la * lb * lb, sizeof(double));
  for (int ey = 0; ey < n; ++ey) {
    for (int qy = 0; qy < q; ++qy) {
      double t = (ey + gx[qy]) * h;
      for (int b = 0; b < la; ++b) {
        vay[qy * la + b] = orc_bspline(ka, nka, ey + b, pa, t);
        day[qy * la + b] = orc_bspline_deriv(ka, nka, ey + b, pa, t);
      }
      for (int b = 0; b < lb; ++b) {
        vby[qy * lb + b] = orc_bspline(kb, nkb, ey + b, pb, t);
        dby[qy * lb + b] = orc_bspline_deriv(kb, nkb, ey + b, pb, t);
      }
    }
    for (int ex = 0; ex < n; ++ex) {
      for (int qx = 0; qx < q; ++qx) {
        double s = (ex + gx[qx]) * h;
        for (int b = 0; b < la; ++b) {
          vax[qx * la + b] = orc_bspline(ka, nka, ex + b, pa, s);
          dax[qx * la + b] = orc_bspline_deriv(ka, nka, ex + b, pa, s);
        }
        for (int b = 0; b < lb; ++b) {
          vbx[qx * lb + b] = orc_bspline(kb, nkb, ex + b, pb, s);
          dbx[qx * lb + b] = orc_bspline_deriv(kb, nkb, ex + b, pb, s);
        }
      }
      memset(em, 0, sizeof(double) * (size_t)la * la * lb * lb);
      memset(ek, 0, sizeof(double) * (size_t)la * la * lb * lb);
      for (int qy = 0; qy < q; ++qy)
        for (int qx = 0; qx < q; ++qx) {
          double s = (ex + gx[qx]) * h, t = (ey + gx[qy]) * h;
          double wq = gw[qx] * gw[qy] * h * h;
          double X[2], J[2][2];
          geom_eval(domain, s, t, X, J);
          double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          double adet = fabs(det);
          /* inverse transpose of J maps parametric to physical gradients */
          double it00 = J[1][1] / det, it01 = -J[1][0] / det;
          double it10 = -J[0][1] / det, it11 = J[0][0] / det;
          for (int by = 0; by < la; ++by)
            for (int bx = 0; bx < la; ++bx) {
              double vx = vax[qx * la + bx], dx = dax[qx * la + bx];
              double vy = vay[qy * la + by], dy = day[qy * la + by];
              double Pi = vx * vy, gs = dx * vy, gt = vx * dy;
              double gX = it00 * gs + it01 * gt, gY = it10 * gs + it11 * gt;
              for (int cy = 0; cy < lb; ++cy)
                for (int cx = 0; cx < lb; ++cx) {
                  double ux = vbx[qx * lb + cx], ddx = dbx[qx * lb + cx];
                  double uy = vby[qy * lb + cy], ddy = dby[qy * lb + cy];
                  size_t e = (((size_t)by * la + bx) * lb + cy) * lb + cx;
                  em[e] += Pi * (ux * uy) * adet * wq;
                  double hs = ddx * uy, ht = ux * ddy;
                  double hX = it00 * hs + it01 * ht, hY = it10 * hs + it11 * ht;
                  ek[e] += (gX * hX + gY * hY) * adet * wq;
                }
            }
        }
      /* scatter the element matrices: local function b of degree pa is global index ex + b */
      for (int by = 0; by < la; ++by)
        for (int bx = 0; bx < la; ++bx) {
          int row = (ey + by) * Na + (ex + bx);
          for (int cy = 0; cy < lb; ++cy)
            for (int cx = 0; cx < lb; ++cx) {
              int col = (ey + cy) * Nb + (ex + cx);
              size_t e = (((size_t)by * la + bx) * lb + cy) * lb + cx;
              if (mass) csr_add(mass, row, col, em[e]);
              if (stiff) csr_add(stiff, row, col, ek[e]);
            }
        }
    }
  }
  free(vax); free(dax); free(vay); free(day);
  free(vbx); free(dbx); free(vby); free(dby);
  free(em); free(ek);
  free(ka);
  free(kb);
  free(gx);
  free(gw);
}

/* Restriction of a full matrix to the interior functions (homogeneous Dirichlet: the first
 * and last function per direction are removed; exact because the basis is interpolatory at
 * both ends).  Interior index ordering is lexicographic with the first direction fastest. */
static void reduce_dirichlet(const ocsr *f, int Na, int Nb, ocsr *r) {
  int na = Na - 2, nb = Nb - 2;
  r->nr = na * na;
  r->nc = nb * nb;
  r->rp = (int *)xcalloc((size_t)r->nr + 1, sizeof(int));
  int cnt = 0;
  for (int iy = 1; iy < Na - 1; ++iy)
    for (int ix = 1; ix < Na - 1; ++ix) {
      int row = iy * Na + ix;
      for (int k = f->rp[row]; k < f->rp[row + 1]; ++k) {
        int c = f->ci[k], cx = c % Nb, cy = c / Nb;
        if (cx >= 1 && cx < Nb - 1 && cy >= 1 && cy < Nb - 1) ++cnt;
      }
    }
  r->nnz = cnt;
  r->ci = (int *)xcalloc((size_t)cnt, sizeof(int));
  r->v = (double *)xcalloc((size_t)cnt, sizeof(double));
  int k2 = 0;
  for (int iy = 1; iy < Na - 1; ++iy)
    for (int ix = 1; ix < Na - 1; ++ix) {
      int row = iy * Na + ix, rr = (iy - 1) * na + (ix - 1);
      r->rp[rr] = k2;
      for (int k = f->rp[row]; k < f->rp[row + 1]; ++k) {
        int c = f->ci[k], cx = c % Nb, cy = c / Nb;
        if (cx >= 1 && cx < Nb - 1 && cy >= 1 && cy < Nb - 1) {
          r->ci[k2] = (cy - 1) * nb + (cx - 1);
          r->v[k2] = f->v[k];
          ++k2;
        }
      }
    }
  r->rp[r->nr] = k2;
}

/* Row-sum lumping M^L_ii = sum_j M_ij over the full row (Sec. 4, after eq:PM), returned for
 * the interior functions only. */
static double *lumped_interior(const ocsr *full, int N) {
  double *d = (double *)xcalloc((size_t)(N - 2) * (N - 2), sizeof(double));
  for (int iy = 1; iy < N - 1; ++iy)
    for (int ix = 1; ix < N - 1; ++ix) {
      int row = iy * N + ix;
      double s = 0.0;
      for (int k = full->rp[row]; k < full->rp[row + 1]; ++k) s += full->v[k];
      d[(iy - 1) * (N - 2) + (ix - 1)] = s;
    }
  return d;
}

/* C = A + c B for CSR matrices on the same pattern */
static void csr_axpby_same(const ocsr *a, double c, const ocsr *b, ocsr *out) {
  out->nr = a->nr;
  out->nc = a->nc;
  out->nnz = a->nnz;
  out->rp = (int *)xcalloc((size_t)a->nr + 1, sizeof(int));
  out->ci = (int *)xcalloc((size_t)a->nnz, sizeof(int));
  out->v = (double *)xcalloc((size_t)a->nnz, sizeof(double));
  memcpy(out->rp, a->rp, sizeof(int) * (size_t)(a->nr + 1));
  memcpy(out->ci, a->ci, sizeof(int) * (size_t)a->nnz);
  for (int k = 0; k < a->nnz; ++k) out->v[k] = a->v[k] + c * b->v[k];
}

/* ------------------------------------------------------------------ */
/* Problem: discretisation at degree p and at p = 1                    */
/* ------------------------------------------------------------------ */

typedef struct {
  int p, n, domain, q;
  int N, Nin, ndof;    /* degree p: functions per direction, interior per direction, dofs */
  int N1, N1in, ndof1; /* degree 1 */
  ocsr Mf, Kf, M, K;   /* degree p mass and stiffness, full and interior */
  ocsr M1f, K1f, M1, K1;
  ocsr Pf, P;          /* P_1^p (rows degree p, cols degree 1), full and interior */
  double *MLp, *ML1;   /* lumped masses on the interior */
} oprob;

ORC_API oprob *orc_problem_create(int p, int n, int domain) {
  if (p < 1 || n < 2 || (domain != 0 && domain != 1)) return NULL;
  oprob *P = (oprob *)xcalloc(1, sizeof(oprob));
  P->p = p;
  P->n = n;
  P->domain = domain;
  P->q = p + 1; /* reading: p+1 Gauss points per direction for every integral */
  P->N = n + p;
  P->Nin = n + p - 2;
  P->ndof = P->Nin * P->Nin;
  P->N1 = n + 1;
  P->N1in = n - 1;
  P->ndof1 = P->N1in * P->N1in;
  assemble_full(domain, n, p, p, P->q, &P->Mf, &P->Kf);
  assemble_full(domain, n, 1, 1, P->q, &P->M1f, &P->K1f);
  assemble_full(domain, n, p, 1, P->q, &P->Pf, NULL);
  reduce_dirichlet(&P->Mf, P->N, P->N, &P->M);
  reduce_dirichlet(&P->Kf, P->N, P->N, &P->K);
  reduce_dirichlet(&P->M1f, P->N1, P->N1, &P->M1);
  reduce_dirichlet(&P->K1f, P->N1, P->N1, &P->K1);
  reduce_dirichlet(&P->Pf, P->N, P->N1, &P->P);
  P->MLp = lumped_interior(&P->Mf, P->N);
  P->ML1 = lumped_interior(&P->M1f, P->N1);
  return P;
}

ORC_API void orc_problem_free(oprob *P) {
  if (!P) return;
  csr_free(&P->Mf);
  csr_free(&P->Kf);
  csr_free(&P->M);
  csr_free(&P->K);
  csr_free(&P->M1f);
  csr_free(&P->K1f);
  csr_free(&P->M1);
  csr_free(&P->K1);
  csr_free(&P->Pf);
  csr_free(&P->P);
  free(P->MLp);
  free(P->ML1);
  free(P);
}

ORC_API void orc_problem_dims(const oprob *P, int *out5) {
  out5[0] = P->N;
  out5[1] = P->Nin;
  out5[2] = P->ndof;
  out5[3] = P->N1in;
  out5[4] = P->ndof1;
}

static const ocsr *pick(const oprob *P, int which) {
  switch (which) {
    case 0: return &P->M;
    case 1: return &P->K;
    case 2: return &P->Mf;
    case 3: return &P->Kf;
    case 4: return &P->M1;
    case 5: return &P->K1;
    case 6: return &P->M1f;
    case 7: return &P->K1f;
    case 8: return &P->P;
    case 9: return &P->Pf;
    default: return NULL;
  }
}

/* shape query: out3 = {rows, cols, nnz} */
ORC_API int orc_matrix_shape(const oprob *P, int which, int *out3) {
  const ocsr *a = pick(P, which);
  if (!a) return -1;
  out3[0] = a->nr;
  out3[1] = a->nc;
  out3[2] = a->nnz;
  return 0;
}

ORC_API int orc_matrix_get(const oprob *P, int which, int *rp, int *ci, double *v) {
  const ocsr *a = pick(P, which);
  if (!a) return -1;
  memcpy(rp, a->rp, sizeof(int) * (size_t)(a->nr + 1));
  memcpy(ci, a->ci, sizeof(int) * (size_t)a->nnz);
  memcpy(v, a->v, sizeof(double) * (size_t)a->nnz);
  return 0;
}

ORC_API void orc_lumped(const oprob *P, double *mlp, double *ml1) {
  memcpy(mlp, P->MLp, sizeof(double) * (size_t)P->ndof);
  memcpy(ml1, P->ML1, sizeof(double) * (size_t)P->ndof1);
}

/* one factor of a source mode: sin(k pi s) for k >= 1; k = 0 stands for the constant 1, so that
 * the paper's own benchmark source f = 1 is the single mode (0, 0, 1) */
static double mode1(int k, double s) { return k == 0 ? 1.0 : sin(k * M_PI * s); }

/* Load vector int f Phi_i dOmega on the interior functions, for
 * f = sum_q amp_q m(k_q, s) m(l_q, t) in parameter coordinates (s,t) (on the unit square these
 * are the physical coordinates), by the same element loop and quadrature. */
ORC_API void orc_load_vector(const oprob *P, int nm, const int *km, const int *lm, const double *amp,
                             double *out) {
  int n = P->n, p = P->p, q = P->q, N = P->N, Nin = P->Nin, nk = n + 2 * p + 1;
  double *kn = (double *)xcalloc((size_t)nk, sizeof(double));
  orc_knots(p, n, kn);
  double *gx = (double *)xcalloc((size_t)q, sizeof(double)), *gw = (double *)xcalloc((size_t)q, sizeof(double));
  orc_gauss(q, gx, gw);
  double *full = (double *)xcalloc((size_t)N * N, sizeof(double));
  double h = 1.0 / n;
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex)
      for (int qy = 0; qy < q; ++qy)
        for (int qx = 0; qx < q; ++qx) {
          double s = (ex + gx[qx]) * h, t = (ey + gx[qy]) * h, wq = gw[qx] * gw[qy] * h * h;
          double X[2], J[2][2];
          geom_eval(P->domain, s, t, X, J);
          double adet = fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
          double f = 0.0;
          for (int m = 0; m < nm; ++m) f += amp[m] * mode1(km[m], s) * mode1(lm[m], t);
          for (int by = 0; by <= p; ++by) {
            double vy = orc_bspline(kn, nk, ey + by, p, t);
            for (int bx = 0; bx <= p; ++bx) {
              double v = orc_bspline(kn, nk, ex + bx, p, s) * vy;
              full[(ey + by) * N + (ex + bx)] += f * v * adet * wq;
            }
          }
        }
  for (int iy = 1; iy < N - 1; ++iy)
    for (int ix = 1; ix < N - 1; ++ix) out[(iy - 1) * Nin + (ix - 1)] = full[iy * N + ix];
  free(full);
  free(kn);
  free(gx);
  free(gw);
}

/* Evaluate the spline with interior coefficients c at parameter point (s,t): only the p+1
 * functions per direction living on the element that contains the point are non-zero. */
ORC_API double orc_eval_spline(const oprob *P, const double *c, double s, double t) {
  int n = P->n, p = P->p, Nin = P->Nin, nk = n + 2 * p + 1;
  double kn[4096];
  if (nk > 4096) return NAN;
  orc_knots(p, n, kn);
  int ex = (int)(s * n), ey = (int)(t * n);
  if (ex > n - 1) ex = n - 1;
  if (ey > n - 1) ey = n - 1;
  if (ex < 0) ex = 0;
  if (ey < 0) ey = 0;
  double u = 0.0;
  for (int iy = ey; iy <= ey + p; ++iy) {
    if (iy < 1 || iy > P->N - 2) continue;
    double vy = orc_bspline(kn, nk, iy, p, t);
    for (int ix = ex; ix <= ex + p; ++ix) {
      if (ix < 1 || ix > P->N - 2) continue;
      u += c[(iy - 1) * Nin + (ix - 1)] * orc_bspline(kn, nk, ix, p, s) * vy;
    }
  }
  return u;
}

/* L2 error || u_h - a * sin(pi s) sin(pi t) ||_{L2(Omega)} with a (2p+2)-point rule per
 * direction, for the manufactured-solution convergence check. */
ORC_API double orc_l2_error_sinsin(const oprob *P, const double *c, double a) {
  int n = P->n, q = 2 * P->p + 2;
  double *gx = (double *)xcalloc((size_t)q, sizeof(double)), *gw = (double *)xcalloc((size_t)q, sizeof(double));
  orc_gauss(q, gx, gw);
  double h = 1.0 / n, e2 = 0.0;
  for (int ey = 0; ey < n; ++ey)
    for (int ex = 0; ex < n; ++ex)
      for (int qy = 0; qy < q; ++qy)
        for (int qx = 0; qx < q; ++qx) {
          double s = (ex + gx[qx]) * h, t = (ey + gx[qy]) * h, wq = gw[qx] * gw[qy] * h * h;
          double X[2], J[2][2];
          geom_eval(P->domain, s, t, X, J);
          double adet = fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
          double d = orc_eval_spline(P, c, s, t) - a * sin(M_PI * X[0]) * sin(M_PI * X[1]);
          e2 += d * d * adet * wq;
        }
  free(gx);
  free(gw);
  return sqrt(e2);
}

/* ------------------------------------------------------------------ */
/* Banded Cholesky: the direct solver                                  */
/* ------------------------------------------------------------------ */

typedef struct {
  int n, bw;
  double *L; /* L[i*(bw+1) + d] = L(i, i-d) */
} oband;

static int band_factor(const ocsr *a, oband *f) {
  int n = a->nr, bw = 0;
  for (int i = 0; i < n; ++i)
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k)
      if (i - a->ci[k] > bw) bw = i - a->ci[k];
  f->n = n;
  f->bw = bw;
  f->L = (double *)xcalloc((size_t)n * (bw + 1), sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
      int j = a->ci[k];
      if (j <= i) f->L[(size_t)i * (bw + 1) + (i - j)] = a->v[k];
    }
  /* textbook column-free Cholesky on the band: for each i, for j = i-bw..i */
  for (int i = 0; i < n; ++i) {
    int j0 = i - bw < 0 ? 0 : i - bw;
    for (int j = j0; j <= i; ++j) {
      double s = f->L[(size_t)i * (bw + 1) + (i - j)];
      int k0 = (i - bw > j - bw ? i - bw : j - bw);
      if (k0 < 0) k0 = 0;
      for (int k = k0; k < j; ++k) s -= f->L[(size_t)i * (bw + 1) + (i - k)] * f->L[(size_t)j * (bw + 1) + (j - k)];
      if (j == i) {
        if (!(s > 0.0)) return -1;
        f->L[(size_t)i * (bw + 1)] = sqrt(s);
      } else {
        f->L[(size_t)i * (bw + 1) + (i - j)] = s / f->L[(size_t)j * (bw + 1)];
      }
    }
  }
  return 0;
}

static void band_solve(const oband *f, const double *b, double *x) {
  int n = f->n, bw = f->bw;
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    int k0 = i - bw < 0 ? 0 : i - bw;
    for (int k = k0; k < i; ++k) s -= f->L[(size_t)i * (bw + 1) + (i - k)] * x[k];
    x[i] = s / f->L[(size_t)i * (bw + 1)];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    int k1 = i + bw > n - 1 ? n - 1 : i + bw;
    for (int k = i + 1; k <= k1; ++k) s -= f->L[(size_t)k * (bw + 1) + (k - i)] * x[k];
    x[i] = s / f->L[(size_t)i * (bw + 1)];
  }
}

static void band_free(oband *f) {
  free(f->L);
  f->L = NULL;
}

/* Direct solve of (M + c K) x = b on the interior of degree p (level 0) -- brute-force check. */
ORC_API int orc_direct_solve(const oprob *P, double c, const double *b, double *x) {
  ocsr A;
  csr_axpby_same(&P->M, c, &P->K, &A);
  oband f;
  int rc = band_factor(&A, &f);
  if (rc == 0) band_solve(&f, b, x);
  band_free(&f);
  csr_free(&A);
  return rc;
}

/* L2 projection onto the spline space with the consistent mass matrix (reading of the
 * projection of the initial condition in Sec. 3): solve M c = int u0 Phi. */
ORC_API int orc_project(const oprob *P, int nm, const int *km, const int *lm, const double *amp, double *c) {
  double *b = (double *)xcalloc((size_t)P->ndof, sizeof(double));
  orc_load_vector(P, nm, km, lm, amp, b);
  int rc = orc_direct_solve(P, 0.0, b, c);
  free(b);
  return rc;
}

/* ------------------------------------------------------------------ */
/* ILUT (Saad's dual threshold incomplete LU)                          */
/* ------------------------------------------------------------------ */

/* Input A (square CSR), drop tolerance tau, and per-row caps: at most lcap[i] entries are
 * kept in the strict lower part of row i of L and at most ucap[i] in the strict upper part of
 * row i of U; the diagonal of U is always kept.  L has a unit diagonal (not stored).
 * Algorithm, row by row:
 *   w := a_i;  tau_i := tau * ||a_i||_2
 *   for k < i in increasing order with w_k != 0:
 *       w_k := w_k / u_kk;  if |w_k| < tau_i drop it, else w := w - w_k * (row k of U, cols > k)
 *   drop every w_j (j != i) with |w_j| < tau_i
 *   keep the lcap[i] largest |w_j|, j < i, as row i of L; u_ii := w_i; keep the ucap[i]
 *   largest |w_j|, j > i, as row i of U  (ties: smaller column first).
 * A non-positive or non-finite pivot u_ii is an error (return -1). */
typedef struct {
  int n;
  ocsr L, U; /* L strict lower; U upper including the diagonal (first entry of each row) */
} oilut;

typedef struct {
  int j;
  double a;
} ent;

static int ent_cmp(const void *x, const void *y) {
  const ent *p = (const ent *)x, *q = (const ent *)y;
  double ap = fabs(p->a), aq = fabs(q->a);
  if (ap > aq) return -1;
  if (ap < aq) return 1;
  return p->j < q->j ? -1 : (p->j > q->j ? 1 : 0);
}

static int ent_col_cmp(const void *x, const void *y) {
  const ent *p = (const ent *)x, *q = (const ent *)y;
  return p->j < q->j ? -1 : (p->j > q->j ? 1 : 0);
}

static int ilut_factor(const ocsr *A, double tau, const int *lcap, const int *ucap, oilut *F) {
  int n = A->nr;
  F->n = n;
  double *w = (double *)xcalloc((size_t)n, sizeof(double));
  char *nz = (char *)xcalloc((size_t)n, 1);
  int *idx = (int *)xcalloc((size_t)n, sizeof(int));
  ent *buf = (ent *)xcalloc((size_t)n, sizeof(ent));
  /* growable row storage */
  size_t capL = (size_t)A->nnz + 16, capU = (size_t)A->nnz + 16;
  F->L.nr = F->L.nc = n;
  F->U.nr = F->U.nc = n;
  F->L.rp = (int *)xcalloc((size_t)n + 1, sizeof(int));
  F->U.rp = (int *)xcalloc((size_t)n + 1, sizeof(int));
  F->L.ci = (int *)xcalloc(capL, sizeof(int));
  F->L.v = (double *)xcalloc(capL, sizeof(double));
  F->U.ci = (int *)xcalloc(capU, sizeof(int));
  F->U.v = (double *)xcalloc(capU, sizeof(double));
  size_t nl = 0, nu = 0;
  int rc = 0;
  for (int i = 0; i < n && rc == 0; ++i) {
    int cnt = 0;
    double an = 0.0;
    for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int j = A->ci[k];
      w[j] = A->v[k];
      if (!nz[j]) {
        nz[j] = 1;
        idx[cnt++] = j;
      }
      an += A->v[k] * A->v[k];
    }
    double taui = tau * sqrt(an);
    /* elimination over k < i in increasing order, including fill created on the way: fill
     * from row k of U only lands in columns > k, so one increasing scan visits it */
    int kmin = i;
    for (int k = A->rp[i]; k < A->rp[i + 1]; ++k)
      if (A->ci[k] < kmin) kmin = A->ci[k];
    for (int k = kmin; k < i; ++k) {
      if (!nz[k] || w[k] == 0.0) continue;
      double ukk = F->U.v[F->U.rp[k]];
      w[k] /= ukk;
      if (fabs(w[k]) < taui) {
        w[k] = 0.0;
        continue;
      }
      double wk = w[k];
      for (int t = F->U.rp[k] + 1; t < F->U.rp[k + 1]; ++t) {
        int j = F->U.ci[t];
        if (!nz[j]) {
          nz[j] = 1;
          w[j] = 0.0;
          idx[cnt++] = j;
        }
        w[j] -= wk * F->U.v[t];
      }
    }
    /* gather lower and upper candidates after the drop rule */
    int nlc = 0;
    for (int t = 0; t < cnt; ++t) {
      int j = idx[t];
      if (j < i && w[j] != 0.0 && fabs(w[j]) >= taui) buf[nlc++] = (ent){j, w[j]};
    }
    qsort(buf, (size_t)nlc, sizeof(ent), ent_cmp);
    int keep = nlc < lcap[i] ? nlc : lcap[i];
    qsort(buf, (size_t)keep, sizeof(ent), ent_col_cmp);
    if (nl + (size_t)keep > capL) {
      capL = 2 * (nl + (size_t)keep);
      F->L.ci = (int *)realloc(F->L.ci, capL * sizeof(int));
      F->L.v = (double *)realloc(F->L.v, capL * sizeof(double));
    }
    for (int t = 0; t < keep; ++t) {
      F->L.ci[nl] = buf[t].j;
      F->L.v[nl] = buf[t].a;
      ++nl;
    }
    double uii = nz[i] ? w[i] : 0.0;
    int nuc = 0;
    for (int t = 0; t < cnt; ++t) {
      int j = idx[t];
      if (j > i && w[j] != 0.0 && fabs(w[j]) >= taui) buf[nuc++] = (ent){j, w[j]};
    }
    qsort(buf, (size_t)nuc, sizeof(ent), ent_cmp);
    keep = nuc < ucap[i] ? nuc : ucap[i];
    qsort(buf, (size_t)keep, sizeof(ent), ent_col_cmp);
    if (nu + (size_t)keep + 1 > capU) {
      capU = 2 * (nu + (size_t)keep + 1);
      F->U.ci = (int *)realloc(F->U.ci, capU * sizeof(int));
      F->U.v = (double *)realloc(F->U.v, capU * sizeof(double));
    }
    F->U.ci[nu] = i;
    F->U.v[nu] = uii;
    ++nu;
    for (int t = 0; t < keep; ++t) {
      F->U.ci[nu] = buf[t].j;
      F->U.v[nu] = buf[t].a;
      ++nu;
    }
    /* row i is complete: its end offsets are needed by the elimination of later rows */
    F->L.rp[i + 1] = (int)nl;
    F->U.rp[i + 1] = (int)nu;
    if (!(uii > 0.0) || !isfinite(uii)) rc = -1;
    for (int t = 0; t < cnt; ++t) {
      w[idx[t]] = 0.0;
      nz[idx[t]] = 0;
    }
  }
  F->L.nnz = (int)nl;
  F->U.nnz = (int)nu;
  free(w);
  free(nz);
  free(idx);
  free(buf);
  return rc;
}

static void ilut_free(oilut *F) {
  csr_free(&F->L);
  csr_free(&F->U);
}

/* caps from A's row structure: "fill = nnz of A" read as at most as many entries per row in
 * L (strict lower) and in U (strict upper) as A has there */
static void caps_from_pattern(const ocsr *A, int *lcap, int *ucap) {
  for (int i = 0; i < A->nr; ++i) {
    int lo = 0, up = 0;
    for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      if (A->ci[k] < i) ++lo;
      if (A->ci[k] > i) ++up;
    }
    lcap[i] = lo;
    ucap[i] = up;
  }
}

/* Apply the ILUT smoother S = (LU)^{-1}: solve L y = r (unit diagonal), then U z = y. */
static void ilut_apply(const oilut *F, const double *r, double *z) {
  int n = F->n;
  for (int i = 0; i < n; ++i) {
    double s = r[i];
    for (int k = F->L.rp[i]; k < F->L.rp[i + 1]; ++k) s -= F->L.v[k] * z[F->L.ci[k]];
    z[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = z[i];
    for (int k = F->U.rp[i] + 1; k < F->U.rp[i + 1]; ++k) s -= F->U.v[k] * z[F->U.ci[k]];
    z[i] = s / F->U.v[F->U.rp[i]];
  }
}

/* Test entry: factor (M + c K) of the problem with drop tolerance tau; capmode 0 = caps from
 * A's pattern, capmode 1 = unlimited.  Returns the factor through getters. */
static oilut g_last_ilut;
static int g_have_ilut = 0;

ORC_API int orc_ilut(const oprob *P, double c, double tau, int capmode, int *nnzLU) {
  if (g_have_ilut) ilut_free(&g_last_ilut);
  g_have_ilut = 0;
  ocsr A;
  csr_axpby_same(&P->M, c, &P->K, &A);
  int *lc = (int *)xcalloc((size_t)A.nr, sizeof(int)), *uc = (int *)xcalloc((size_t)A.nr, sizeof(int));
  if (capmode == 0)
    caps_from_pattern(&A, lc, uc);
  else
    for (int i = 0; i < A.nr; ++i) lc[i] = uc[i] = A.nr;
  int rc = ilut_factor(&A, tau, lc, uc, &g_last_ilut);
  g_have_ilut = 1;
  nnzLU[0] = g_last_ilut.L.nnz;
  nnzLU[1] = g_last_ilut.U.nnz;
  free(lc);
  free(uc);
  csr_free(&A);
  return rc;
}

ORC_API void orc_ilut_get(int *Lrp, int *Lci, double *Lv, int *Urp, int *Uci, double *Uv) {
  if (!g_have_ilut) return;
  const oilut *F = &g_last_ilut;
  memcpy(Lrp, F->L.rp, sizeof(int) * (size_t)(F->n + 1));
  memcpy(Lci, F->L.ci, sizeof(int) * (size_t)F->L.nnz);
  memcpy(Lv, F->L.v, sizeof(double) * (size_t)F->L.nnz);
  memcpy(Urp, F->U.rp, sizeof(int) * (size_t)(F->n + 1));
  memcpy(Uci, F->U.ci, sizeof(int) * (size_t)F->U.nnz);
  memcpy(Uv, F->U.v, sizeof(double) * (size_t)F->U.nnz);
}

/* ------------------------------------------------------------------ */
/* p-multigrid (Sec. 4)                                                */
/* ------------------------------------------------------------------ */

/* Per time level: A_{h,p} = M + kappa dt K; ILUT(A); A_{h,1} = M_1 + kappa dt K_1 factored. */
typedef struct {
  const oprob *P;
  double dt;
  ocsr A;
  oilut S;
  oband A1;
  int nu1, nu2;
  double tol;   /* spatial stop: ||b - A x|| <= tol ||b|| */
  int maxcyc;
  long long cycles; /* V-cycles spent */
  long long solves;
  int failed;
  double *r, *z, *r1, *e1, *t; /* work */
} opmg;

static int pmg_init(opmg *G, const oprob *P, double kappa, double dt, double tau, int nu1, int nu2, double tol,
                    int maxcyc) {
  memset(G, 0, sizeof(*G));
  G->P = P;
  G->dt = dt;
  G->nu1 = nu1;
  G->nu2 = nu2;
  G->tol = tol;
  G->maxcyc = maxcyc;
  csr_axpby_same(&P->M, kappa * dt, &P->K, &G->A);
  int *lc = (int *)xcalloc((size_t)G->A.nr, sizeof(int)), *uc = (int *)xcalloc((size_t)G->A.nr, sizeof(int));
  caps_from_pattern(&G->A, lc, uc);
  int rc = ilut_factor(&G->A, tau, lc, uc, &G->S);
  free(lc);
  free(uc);
  if (rc) return -4;
  /* coarse operator: the same problem rediscretised at p = 1 with the same dt */
  ocsr A1;
  csr_axpby_same(&P->M1, kappa * dt, &P->K1, &A1);
  rc = band_factor(&A1, &G->A1);
  csr_free(&A1);
  if (rc) return -4;
  G->r = (double *)xcalloc((size_t)P->ndof, sizeof(double));
  G->z = (double *)xcalloc((size_t)P->ndof, sizeof(double));
  G->t = (double *)xcalloc((size_t)P->ndof, sizeof(double));
  G->r1 = (double *)xcalloc((size_t)P->ndof1, sizeof(double));
  G->e1 = (double *)xcalloc((size_t)P->ndof1, sizeof(double));
  return 0;
}

static void pmg_free(opmg *G) {
  csr_free(&G->A);
  ilut_free(&G->S);
  band_free(&G->A1);
  free(G->r);
  free(G->z);
  free(G->t);
  free(G->r1);
  free(G->e1);
}

/* r = b - A x */
static void residual(const ocsr *A, const double *b, const double *x, double *r) {
  csr_mv(A, x, r);
  for (int i = 0; i < A->nr; ++i) r[i] = b[i] - r[i];
}

/* One p-multigrid V-cycle on A x = b (Sec. 4, steps 1-5). */
static void pmg_vcycle(opmg *G, const double *b, double *x) {
  const oprob *P = G->P;
  int n = P->ndof, n1 = P->ndof1;
  /* 1. nu1 pre-smoothing steps x := x + S (b - A x), eq:smooth */
  for (int m = 0; m < G->nu1; ++m) {
    residual(&G->A, b, x, G->r);
    ilut_apply(&G->S, G->r, G->z);
    for (int i = 0; i < n; ++i) x[i] += G->z[i];
  }
  /* 2. residual restricted to p = 1: r_1 = (M_1^L)^{-1} P_p^1 (b - A x), P_p^1 = (P_1^p)^T */
  residual(&G->A, b, x, G->r);
  csr_mtv(&P->P, G->r, G->r1);
  for (int j = 0; j < n1; ++j) G->r1[j] /= P->ML1[j];
  /* 3. residual equation A_{h,1} e_1 = r_1 solved directly, eq:res */
  band_solve(&G->A1, G->r1, G->e1);
  /* 4. prolongation and update x := x + (M_p^L)^{-1} P_1^p e_1, eq:prolongation */
  csr_mv(&P->P, G->e1, G->t);
  for (int i = 0; i < n; ++i) x[i] += G->t[i] / P->MLp[i];
  /* 5. nu2 post-smoothing steps */
  for (int m = 0; m < G->nu2; ++m) {
    residual(&G->A, b, x, G->r);
    ilut_apply(&G->S, G->r, G->z);
    for (int i = 0; i < n; ++i) x[i] += G->z[i];
  }
}

/* Spatial solve: V-cycles from the initial guess in x until ||b - A x||_2 <= tol ||b||_2
 * (reading: relative to the right-hand side) or maxcyc cycles. */
static int pmg_solve(opmg *G, const double *b, double *x) {
  int n = G->P->ndof;
  double bn = nrm2(n, b);
  G->solves++;
  if (bn == 0.0) {
    /* a zero right-hand side has the exact solution x = 0 (a relative stop test cannot be met
     * from a non-zero guess) */
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    return 0;
  }
  for (int c = 0;; ++c) {
    residual(&G->A, b, x, G->r);
    double rn = nrm2(n, G->r);
    if (!isfinite(rn)) {
      G->failed = 1;
      return -7;
    }
    if (rn <= G->tol * bn) return 0;
    if (c >= G->maxcyc) {
      G->failed = 1;
      return -5;
    }
    pmg_vcycle(G, b, x);
    G->cycles++;
  }
}

/* Test entry: solve (M + kappa dt K) x = b by p-multigrid from guess x. */
ORC_API int orc_pmg_solve(const oprob *P, double kappa, double dt, double tau, int nu1, int nu2, double tol,
                          int maxcyc, const double *b, double *x, int *cycles) {
  opmg G;
  int rc = pmg_init(&G, P, kappa, dt, tau, nu1, nu2, tol, maxcyc);
  if (rc == 0) rc = pmg_solve(&G, b, x);
  *cycles = (int)G.cycles;
  pmg_free(&G);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Time stepping (Sec. 2, eq:los with theta = 1; Sec. 3, eq:mgrit)      */
/* ------------------------------------------------------------------ */

/* source time factor: kind 0 -> 1, kind 1 -> exp(-t) */
static double tfac(int kind, double t) { return kind == 1 ? exp(-t) : 1.0; }

/* Sequential implicit Euler with direct solves:
 *   U_0 = u0;  (M + kappa dt K) U_{k+1} = M U_k + dt s(t_{k+1}) F,  k = 0..Nt-1,
 * i.e. the block forward solve of A u = g in eq:mgrit.  U is (Nt+1) x ndof, row-major. */
ORC_API int orc_sequential(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind,
                           const double *u0, double *U) {
  int n = P->ndof;
  double dt = T / Nt;
  ocsr A;
  csr_axpby_same(&P->M, kappa * dt, &P->K, &A);
  oband f;
  int rc = band_factor(&A, &f);
  csr_free(&A);
  if (rc) return -4;
  double *rhs = (double *)xcalloc((size_t)n, sizeof(double));
  memcpy(U, u0, sizeof(double) * (size_t)n);
  for (int k = 0; k < Nt; ++k) {
    csr_mv(&P->M, U + (size_t)k * n, rhs);
    double c = dt * tfac(tkind, (k + 1) * dt);
    for (int i = 0; i < n; ++i) rhs[i] += c * F[i];
    band_solve(&f, rhs, U + (size_t)(k + 1) * n);
  }
  free(rhs);
  band_free(&f);
  return 0;
}

/* Sequential implicit Euler with p-multigrid spatial solves (guess: previous step). */
ORC_API int orc_sequential_pmg(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind,
                               const double *u0, double tau, double stol, int maxcyc, double *U,
                               long long *cycles) {
  int n = P->ndof;
  double dt = T / Nt;
  opmg G;
  int rc = pmg_init(&G, P, kappa, dt, tau, 1, 1, stol, maxcyc);
  if (rc) {
    pmg_free(&G);
    return rc;
  }
  double *rhs = (double *)xcalloc((size_t)n, sizeof(double));
  memcpy(U, u0, sizeof(double) * (size_t)n);
  for (int k = 0; k < Nt && rc == 0; ++k) {
    csr_mv(&P->M, U + (size_t)k * n, rhs);
    double c = dt * tfac(tkind, (k + 1) * dt);
    for (int i = 0; i < n; ++i) rhs[i] += c * F[i];
    memcpy(U + (size_t)(k + 1) * n, U + (size_t)k * n, sizeof(double) * (size_t)n);
    rc = pmg_solve(&G, rhs, U + (size_t)(k + 1) * n);
  }
  *cycles = G.cycles;
  free(rhs);
  pmg_free(&G);
  return rc;
}

/* ------------------------------------------------------------------ */
/* MGRIT (Sec. 3)                                                      */
/* ------------------------------------------------------------------ */

/* Level l of the time hierarchy: N_l intervals of size dt_l = m^l dt (rediscretised,
 * Sec. 3), the vector v (u at level 0, the correction at coarser levels) and the
 * right-hand side g of A^{(l)} v = g^{(l)} at coarse levels.  The step of A^{(l)} is
 *   level 0:  v_{k+1} = Psi_0 (M v_k + dt_0 s(t_{k+1}) F)      (one spatial solve)
 *   level l:  v_{k+1} = Psi_l M v_k + g_{k+1}                   (Psi_l = (M + kappa dt_l K)^{-1})
 * and the residual of A^{(l)} v = g at point k is step(v_{k-1}) - v_k. */
typedef struct {
  int Nl;
  double dt;
  opmg G;
  double *v, *g;
} olev;

typedef struct {
  const oprob *P;
  double kappa, T;
  int Nt, m, nlev, guess;
  const double *F;
  int tkind;
  olev *L;
  double *b, *x; /* work */
  int rc;
} omgrit;

/* one step at level l from v[k] to target k+1, written into out (which may alias v[k+1]).
 * guess policy: 0 zero, 1 previous point, 2 current value of the target at level 0 (it carries
 * the previous MGRIT iterate) and the previous point at coarser levels (whose state restarts
 * from zero in every cycle, so their targets carry no information in the first sweeps). */
static void mg_step(omgrit *S, int l, int k, double *out) {
  olev *L = &S->L[l];
  int n = S->P->ndof;
  const double *vk = L->v + (size_t)k * n;
  csr_mv(&S->P->M, vk, S->b);
  if (l == 0) {
    double c = L->dt * tfac(S->tkind, (k + 1) * L->dt);
    for (int i = 0; i < n; ++i) S->b[i] += c * S->F[i];
  }
  const double *tgt = L->v + (size_t)(k + 1) * n;
  const double *gk = l > 0 ? L->g + (size_t)(k + 1) * n : NULL; /* coarse right-hand side, added after the solve */
  for (int i = 0; i < n; ++i) {
    if (S->guess == 0)
      S->x[i] = 0.0;
    else if (S->guess == 1 || l > 0)
      S->x[i] = vk[i];
    else
      S->x[i] = tgt[i];
  }
  int rc = pmg_solve(&L->G, S->b, S->x);
  if (rc && !S->rc) S->rc = rc;
  for (int i = 0; i < n; ++i) out[i] = S->x[i] + (gk ? gk[i] : 0.0);
}

/* F-relaxation: inside every coarse interval propagate from its C-point to its F-points. */
static void f_relax(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof, m = S->m;
  for (int j = 0; j * m < L->Nl; ++j)
    for (int s = 1; s < m && j * m + s <= L->Nl; ++s) {
      int k = j * m + s - 1;
      mg_step(S, l, k, L->v + (size_t)(k + 1) * n);
    }
}

/* C-relaxation: every C-point j m (j >= 1) from its preceding F-point. */
static void c_relax(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof, m = S->m;
  for (int j = 1; j * m <= L->Nl; ++j) mg_step(S, l, j * m - 1, L->v + (size_t)(j * m) * n);
}

/* residual at the C-points after relaxation, r_j = step(v_{jm-1}) - v_{jm}, injected as the
 * right-hand side of level l+1 (its point j).  Returns sum_j ||r_j||^2. */
static double c_residual_inject(omgrit *S, int l) {
  olev *L = &S->L[l], *C = &S->L[l + 1];
  int n = S->P->ndof, m = S->m;
  double *tmp = (double *)xcalloc((size_t)n, sizeof(double));
  double s2 = 0.0;
  memset(C->g, 0, sizeof(double) * (size_t)n); /* point 0 is exact: zero residual */
  for (int j = 1; j * m <= L->Nl; ++j) {
    mg_step(S, l, j * m - 1, tmp);
    double *gj = C->g + (size_t)j * n;
    const double *vj = L->v + (size_t)(j * m) * n;
    for (int i = 0; i < n; ++i) {
      gj[i] = tmp[i] - vj[i];
      s2 += gj[i] * gj[i];
    }
  }
  free(tmp);
  return s2;
}

/* coarsest level: block forward solve of A^{(L)} v = g (sequential time stepping) */
static void coarsest_solve(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof;
  memcpy(L->v, L->g, sizeof(double) * (size_t)n);
  for (int k = 0; k < L->Nl; ++k) mg_step(S, l, k, L->v + (size_t)(k + 1) * n);
}

/* the MGRIT recursion (Sec. 3): at level l < L: FCF-relaxation, injected residual, recurse,
 * update v := v + P v^{(l+1)} with ideal interpolation = correct C-points then F-relax. */
static double mgrit_cycle(omgrit *S, int l, int do_interp) {
  if (l == S->nlev - 1) {
    coarsest_solve(S, l);
    return 0.0;
  }
  olev *L = &S->L[l], *C = &S->L[l + 1];
  int n = S->P->ndof, m = S->m;
  f_relax(S, l);
  c_relax(S, l);
  f_relax(S, l);
  double r2 = c_residual_inject(S, l);
  if (l == 0) {
    /* level 0 convergence decision is taken by the caller before the coarse correction */
    return r2;
  }
  memset(C->v, 0, sizeof(double) * (size_t)(C->Nl + 1) * n);
  mgrit_cycle(S, l + 1, 1);
  for (int j = 1; j * m <= L->Nl; ++j) {
    double *vj = L->v + (size_t)(j * m) * n;
    const double *ej = C->v + (size_t)j * n;
    for (int i = 0; i < n; ++i) vj[i] += ej[i];
  }
  if (do_interp) f_relax(S, l);
  return r2;
}

/* MGRIT on level 0.  Hierarchy: N_l = N_t / m^l, coarsening stops at level max_levels-1 or
 * when N_l <= coarsest_max.  Initial guess: U_0 = u0, U_k = 0 for k >= 1 (reading).
 * Stop when ||r^{(k)}|| <= tol ||r^{(0)}|| with r the level-0 C-point residual after
 * FCF-relaxation (reading of the relative residual criterion of Sec. 5).  The converged
 * iterate is the post-FCF state, whose F-points are already consistent.
 * Spatial solves stop at stol on level 0 and at ctol on the coarse levels (ctol <= 0: stol).
 * The paper fixes neither; the coarse levels only supply corrections, so their tolerance
 * changes the convergence rate, not the fixed point that the level-0 test measures.
 * out: iters, V-cycles, spatial solves; res_hist (up to 200 entries, relative). */
ORC_API int orc_mgrit(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind, const double *u0,
                      int m, int max_levels, int coarsest_max, double tol, int max_iter, double tau, double stol,
                      double ctol, int maxcyc, int guess, double *U, int *iters, long long *cycles,
                      long long *solves, double *res_hist) {
  int n = P->ndof;
  omgrit S;
  memset(&S, 0, sizeof(S));
  S.P = P;
  S.kappa = kappa;
  S.T = T;
  S.Nt = Nt;
  S.m = m;
  S.F = F;
  S.tkind = tkind;
  S.guess = guess;
  int nlev = 1;
  {
    int Nl = Nt;
    while (nlev < max_levels && Nl > coarsest_max && Nl / m >= 1) {
      Nl /= m;
      ++nlev;
    }
  }
  S.nlev = nlev;
  S.L = (olev *)xcalloc((size_t)nlev, sizeof(olev));
  int Nl = Nt;
  double dt = T / Nt;
  int rc = 0;
  for (int l = 0; l < nlev; ++l) {
    S.L[l].Nl = Nl;
    S.L[l].dt = dt;
    if (rc == 0) rc = pmg_init(&S.L[l].G, P, kappa, dt, tau, 1, 1, (l > 0 && ctol > 0) ? ctol : stol, maxcyc);
    S.L[l].v = l == 0 ? U : (double *)xcalloc((size_t)(Nl + 1) * n, sizeof(double));
    S.L[l].g = l == 0 ? NULL : (double *)xcalloc((size_t)(Nl + 1) * n, sizeof(double));
    Nl /= m;
    dt *= m;
  }
  S.b = (double *)xcalloc((size_t)n, sizeof(double));
  S.x = (double *)xcalloc((size_t)n, sizeof(double));
  int it = 0;
  if (rc == 0) {
    memset(U, 0, sizeof(double) * (size_t)(Nt + 1) * n);
    memcpy(U, u0, sizeof(double) * (size_t)n);
    if (nlev == 1) {
      /* no coarsening possible: sequential solve at level 0 */
      for (int k = 0; k < Nt; ++k) mg_step(&S, 0, k, U + (size_t)(k + 1) * n);
    } else {
      double r0 = -1.0;
      for (;;) {
        double r2 = mgrit_cycle(&S, 0, 0);
        double rn = sqrt(r2);
        if (r0 < 0.0) r0 = rn;
        double rel = r0 > 0.0 ? rn / r0 : 0.0;
        if (res_hist && it < 200) res_hist[it] = rel;
        if (S.rc) break;
        if (!isfinite(rn)) {
          rc = -7;
          break;
        }
        if (rn <= tol * r0 || r0 == 0.0) break;
        if (it >= max_iter) {
          rc = -6;
          break;
        }
        /* coarse correction from the injected residual, then the next FCF */
        olev *C = &S.L[1];
        memset(C->v, 0, sizeof(double) * (size_t)(C->Nl + 1) * n);
        mgrit_cycle(&S, 1, 1);
        for (int j = 1; j * m <= Nt; ++j) {
          double *vj = U + (size_t)(j * m) * n;
          const double *ej = C->v + (size_t)j * n;
          for (int i = 0; i < n; ++i) vj[i] += ej[i];
        }
        ++it;
      }
    }
  }
  if (rc == 0 && S.rc) rc = S.rc;
  long long cyc = 0, sol = 0;
  for (int l = 0; l < nlev; ++l) {
    cyc += S.L[l].G.cycles;
    sol += S.L[l].G.solves;
    pmg_free(&S.L[l].G);
    if (l > 0) {
      free(S.L[l].v);
      free(S.L[l].g);
    }
  }
  *iters = it;
  *cycles = cyc;
  *solves = sol;
  free(S.L);
  free(S.b);
  free(S.x);
  return rc;
}
