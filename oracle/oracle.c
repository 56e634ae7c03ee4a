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
 *   - the theta-scheme system of each time step (Sec. 2, eq:los),
 *   - ILUT (Saad's dual-threshold incomplete LU; the smoother named in Sec. 4),
 *   - the p-multigrid V-cycle, steps 1-5, with L2-projection transfers built from the
 *     row-sum-lumped mass matrices (Sec. 4, eq:prolongation, eq:PM), in FP64 or as an FP32
 *     V-cycle inside FP64 iterative refinement,
 *   - at p = 1 an exact (banded Cholesky) solve, or the paper's one h-multigrid W-cycle with
 *     Gauss-Seidel smoothing, canonical prolongation, weighted restriction and a direct solve on
 *     the coarsest mesh (Sec. 4, the paragraph after step 5),
 *   - conjugate gradients preconditioned by the diagonal, the paper's comparison solver (Sec. 4),
 *   - sequential time stepping with direct solves (the block forward solve of eq:mgrit),
 *   - two-level and multilevel MGRIT with FCF-relaxation, injection and ideal interpolation
 *     (Sec. 3, eq:mgrit_coarse and the MGRIT recursion), in V-, W- and F-cycles; the independent
 *     intervals of a sweep may run on several threads (OpenMP), which changes no arithmetic.
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

/* Functions of the physical coordinates (x, y) = F(s, t), for manufactured solutions on the
 * mapped geometry: the load vector int f Phi_i dOmega on the interior functions by the element
 * loop with the (p+1)-point rule, and the L2 error || u_h - u ||_{L2(Omega)} with a (2p+2)-point
 * rule. */
typedef double (*orc_fn2)(double x, double y);

ORC_API void orc_load_vector_fn(const oprob *P, orc_fn2 f, double *out) {
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
          double fv = f(X[0], X[1]);
          for (int by = 0; by <= p; ++by) {
            double vy = orc_bspline(kn, nk, ey + by, p, t);
            for (int bx = 0; bx <= p; ++bx)
              full[(ey + by) * N + (ex + bx)] += fv * orc_bspline(kn, nk, ex + bx, p, s) * vy * adet * wq;
          }
        }
  for (int iy = 1; iy < N - 1; ++iy)
    for (int ix = 1; ix < N - 1; ++ix) out[(iy - 1) * Nin + (ix - 1)] = full[iy * N + ix];
  free(full);
  free(kn);
  free(gx);
  free(gw);
}

ORC_API double orc_l2_error_fn(const oprob *P, const double *c, orc_fn2 u) {
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
          double d = orc_eval_spline(P, c, s, t) - u(X[0], X[1]);
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
/* sparse helpers                                                      */
/* ------------------------------------------------------------------ */

/* r = b - A x */
static void residual(const ocsr *A, const double *b, const double *x, double *r) {
  csr_mv(A, x, r);
  for (int i = 0; i < A->nr; ++i) r[i] = b[i] - r[i];
}

static int int_cmp(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* C = A B, row by row (Gustavson), columns sorted */
static void csr_matmul(const ocsr *a, const ocsr *b, ocsr *c) {
  int nr = a->nr, nc = b->nc;
  double *acc = (double *)xcalloc((size_t)nc, sizeof(double));
  int *mark = (int *)xcalloc((size_t)nc, sizeof(int));
  int *cols = (int *)xcalloc((size_t)nc, sizeof(int));
  size_t cap = (size_t)a->nnz + (size_t)b->nnz + 16, nnz = 0;
  c->nr = nr;
  c->nc = nc;
  c->rp = (int *)xcalloc((size_t)nr + 1, sizeof(int));
  c->ci = (int *)xcalloc(cap, sizeof(int));
  c->v = (double *)xcalloc(cap, sizeof(double));
  for (int i = 0; i < nr; ++i) {
    int cnt = 0;
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
      int j = a->ci[k];
      for (int t = b->rp[j]; t < b->rp[j + 1]; ++t) {
        int col = b->ci[t];
        if (mark[col] != i + 1) {
          mark[col] = i + 1;
          acc[col] = 0.0;
          cols[cnt++] = col;
        }
        acc[col] += a->v[k] * b->v[t];
      }
    }
    qsort(cols, (size_t)cnt, sizeof(int), int_cmp);
    if (nnz + (size_t)cnt > cap) {
      cap = 2 * (nnz + (size_t)cnt);
      c->ci = (int *)realloc(c->ci, cap * sizeof(int));
      c->v = (double *)realloc(c->v, cap * sizeof(double));
    }
    for (int t = 0; t < cnt; ++t) {
      c->ci[nnz] = cols[t];
      c->v[nnz] = acc[cols[t]];
      ++nnz;
    }
    c->rp[i + 1] = (int)nnz;
  }
  c->nnz = (int)nnz;
  free(acc);
  free(mark);
  free(cols);
}

/* T = A^T */
static void csr_transpose(const ocsr *a, ocsr *t) {
  t->nr = a->nc;
  t->nc = a->nr;
  t->nnz = a->nnz;
  t->rp = (int *)xcalloc((size_t)t->nr + 1, sizeof(int));
  t->ci = (int *)xcalloc((size_t)a->nnz, sizeof(int));
  t->v = (double *)xcalloc((size_t)a->nnz, sizeof(double));
  for (int k = 0; k < a->nnz; ++k) t->rp[a->ci[k] + 1]++;
  for (int j = 0; j < t->nr; ++j) t->rp[j + 1] += t->rp[j];
  int *pos = (int *)xcalloc((size_t)t->nr, sizeof(int));
  for (int j = 0; j < t->nr; ++j) pos[j] = t->rp[j];
  for (int i = 0; i < a->nr; ++i)
    for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
      int q = pos[a->ci[k]]++;
      t->ci[q] = i;
      t->v[q] = a->v[k];
    }
  free(pos);
}

static void csr_copy(const ocsr *a, ocsr *c) { csr_axpby_same(a, 0.0, a, c); }

/* ------------------------------------------------------------------ */
/* h-multigrid at p = 1: one W-cycle as the coarse solve (Sec. 4)      */
/* ------------------------------------------------------------------ */

/* The p = 1 space on n elements per direction is coarsened by halving the mesh while the
 * element count is even and larger than 4 (reading: the coarsest mesh has at most 4 elements per
 * direction, or an odd number); the coarsest operator is solved directly. */
#define OHMG_MAX 16

static int hmg_levels(int n, int *ne) {
  int nl = 0;
  for (;;) {
    ne[nl++] = n;
    if (nl == OHMG_MAX || n % 2 != 0 || n <= 4) break;
    n /= 2;
  }
  return nl;
}

typedef struct {
  int nlev;
  int ne[OHMG_MAX];  /* elements per direction of h-level k */
  ocsr A[OHMG_MAX];  /* A[0] = A_{h,1}; A[k] = R[k] A[k-1] P[k] (Galerkin) */
  ocsr P[OHMG_MAX];  /* P[k], k >= 1: canonical prolongation from h-level k to h-level k - 1 */
  ocsr R[OHMG_MAX];  /* R[k] = P[k]^T, the weighted restriction */
  oband C;           /* Cholesky factor of the coarsest operator */
} ohmg;

/* weight of the coarse hat function J (node 2J of the fine grid) in the fine hat function i */
static double hat_weight(int i, int J) {
  int d = i - 2 * J;
  return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0);
}

/* Canonical prolongation of the degree-1 spline space on nf / 2 elements into the one on nf
 * elements, interior functions, both directions: the coarse function is written in the fine basis
 * (a coarse hat is the fine hat at the same node plus half of each fine neighbour); the 2D
 * operator is the tensor product of the 1D ones.  The geometry map does not enter: the spaces are
 * defined on the parameter domain. */
static void hmg_prolong(int nf, ocsr *P) {
  int n1f = nf - 1, n1c = nf / 2 - 1;
  P->nr = n1f * n1f;
  P->nc = n1c * n1c;
  P->rp = (int *)xcalloc((size_t)P->nr + 1, sizeof(int));
  P->ci = (int *)xcalloc((size_t)P->nr * 4 + 1, sizeof(int));
  P->v = (double *)xcalloc((size_t)P->nr * 4 + 1, sizeof(double));
  int k = 0;
  for (int iy = 1; iy <= n1f; ++iy)
    for (int ix = 1; ix <= n1f; ++ix) {
      int row = (iy - 1) * n1f + (ix - 1);
      P->rp[row] = k;
      for (int Jy = (iy - 1) / 2; Jy <= (iy + 1) / 2; ++Jy) {
        double wy = (Jy >= 1 && Jy <= n1c) ? hat_weight(iy, Jy) : 0.0;
        if (wy == 0.0) continue;
        for (int Jx = (ix - 1) / 2; Jx <= (ix + 1) / 2; ++Jx) {
          double wx = (Jx >= 1 && Jx <= n1c) ? hat_weight(ix, Jx) : 0.0;
          if (wx == 0.0) continue;
          P->ci[k] = (Jy - 1) * n1c + (Jx - 1);
          P->v[k] = wy * wx;
          ++k;
        }
      }
    }
  P->rp[P->nr] = k;
  P->nnz = k;
}

static int hmg_init(ohmg *H, int n, const ocsr *A1) {
  memset(H, 0, sizeof(*H));
  H->nlev = hmg_levels(n, H->ne);
  csr_copy(A1, &H->A[0]);
  for (int k = 1; k < H->nlev; ++k) {
    hmg_prolong(H->ne[k - 1], &H->P[k]);
    csr_transpose(&H->P[k], &H->R[k]);
    ocsr AP;
    csr_matmul(&H->A[k - 1], &H->P[k], &AP);
    csr_matmul(&H->R[k], &AP, &H->A[k]);
    csr_free(&AP);
  }
  return band_factor(&H->A[H->nlev - 1], &H->C);
}

static void hmg_free(ohmg *H) {
  for (int k = 0; k < H->nlev; ++k) {
    csr_free(&H->A[k]);
    if (k > 0) {
      csr_free(&H->P[k]);
      csr_free(&H->R[k]);
    }
  }
  band_free(&H->C);
  H->nlev = 0;
}

/* One Gauss-Seidel sweep on A x = b (A on the interior nodes of an n1 x n1 grid, first index
 * fastest) in the four-colour order of the 9-point stencil: the colour of node (ix, iy) is
 * (ix mod 2) + 2 (iy mod 2); colours 0, 1, 2, 3 in turn (dir > 0) or 3, 2, 1, 0 (dir < 0).  Nodes of
 * one colour never couple, so every node update uses the newest values of all its neighbours
 * (reading: the paper names Gauss-Seidel without an ordering). */
static void gs_sweep(const ocsr *A, int n1, const double *b, double *x, int dir) {
  for (int cc = 0; cc < 4; ++cc) {
    int col = dir > 0 ? cc : 3 - cc;
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        if ((ix % 2) + 2 * (iy % 2) != col) continue;
        int i = iy * n1 + ix;
        double s = b[i], d = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) {
          if (A->ci[k] == i)
            d = A->v[k];
          else
            s -= A->v[k] * x[A->ci[k]];
        }
        x[i] = s / d;
      }
  }
}

/* One W-cycle of h-multigrid on A[k] x = b (Sec. 4, the paragraph after step 5): a forward
 * Gauss-Seidel sweep, the residual restricted with R, the level-(k+1) correction from zero by two
 * W-cycles (the coarsest level is solved directly, once), prolongation of the correction, a
 * backward Gauss-Seidel sweep (reading: one pre- and one post-smoothing sweep, the post-sweep in
 * reverse colour order).  wr, wb, wx: work vectors per level. */
static void hmg_wcycle(const ohmg *H, int k, const double *b, double *x, double **wr, double **wb, double **wx) {
  if (k == H->nlev - 1) {
    band_solve(&H->C, b, x);
    return;
  }
  int n = H->A[k].nr, nc = H->A[k + 1].nr, n1 = H->ne[k] - 1;
  gs_sweep(&H->A[k], n1, b, x, +1);
  residual(&H->A[k], b, x, wr[k]);
  csr_mv(&H->R[k + 1], wr[k], wb[k + 1]);
  for (int i = 0; i < nc; ++i) wx[k + 1][i] = 0.0;
  hmg_wcycle(H, k + 1, wb[k + 1], wx[k + 1], wr, wb, wx);
  if (k + 1 < H->nlev - 1) hmg_wcycle(H, k + 1, wb[k + 1], wx[k + 1], wr, wb, wx);
  csr_mv(&H->P[k + 1], wx[k + 1], wr[k]);
  for (int i = 0; i < n; ++i) x[i] += wr[k][i];
  gs_sweep(&H->A[k], n1, b, x, -1);
}

/* ------------------------------------------------------------------ */
/* spatial solvers (Sec. 4): p-multigrid, or Jacobi-preconditioned CG  */
/* ------------------------------------------------------------------ */

#define OMAXLEV 32

/* One time level's spatial operator, theta-scheme (Sec. 2, eq:los):
 *   A = M + theta kappa dt K   (left-hand side, solved by the spatial solver)
 *   B = M - (1 - theta) kappa dt K   (applied to the previous point)
 * solver 0: p-multigrid with ILUT(A) smoothing and, at p = 1, A_{h,1} = M_1 + theta kappa dt K_1
 * (rediscretised) solved exactly (coarse 0, banded Cholesky) or by one h-multigrid W-cycle
 * (coarse 1); prec 1 runs the V-cycle in FP32 inside FP64 iterative refinement (FP64 residual,
 * update and p = 1 solve).  solver 1: conjugate gradients preconditioned by diag(A). */
typedef struct {
  const oprob *P;
  double dt, theta;
  ocsr A, B;
  oilut S;
  oband A1;
  ohmg H;
  double *dg;                         /* diag(A) (solver 1) */
  float *Af, *Lf, *Uf, *Pf;           /* FP32 values on the patterns of A, L, U, P (prec 1) */
  float *imlp, *iml1;                 /* FP32 inverse lumped masses (prec 1) */
  int nu1, nu2, prec, coarse, solver;
  double tol;
  int maxcyc;
} opmg;

/* work vectors of one thread, and its counters per MGRIT level */
typedef struct {
  double *r, *z, *t, *r1, *e1, *b, *x, *q, *out;
  float *rf, *df, *tf, *zf, *r1f;
  double *hr[OHMG_MAX], *hb[OHMG_MAX], *hx[OHMG_MAX];
  long long cyc[OMAXLEV], sol[OMAXLEV];
} owork;

static void work_init(owork *w, const oprob *P) {
  memset(w, 0, sizeof(*w));
  size_t n = (size_t)P->ndof, n1 = (size_t)P->ndof1;
  w->r = (double *)xcalloc(n, sizeof(double));
  w->z = (double *)xcalloc(n, sizeof(double));
  w->t = (double *)xcalloc(n, sizeof(double));
  w->b = (double *)xcalloc(n, sizeof(double));
  w->x = (double *)xcalloc(n, sizeof(double));
  w->q = (double *)xcalloc(n, sizeof(double));
  w->out = (double *)xcalloc(n, sizeof(double));
  w->r1 = (double *)xcalloc(n1, sizeof(double));
  w->e1 = (double *)xcalloc(n1, sizeof(double));
  w->rf = (float *)xcalloc(n, sizeof(float));
  w->df = (float *)xcalloc(n, sizeof(float));
  w->tf = (float *)xcalloc(n, sizeof(float));
  w->zf = (float *)xcalloc(n, sizeof(float));
  w->r1f = (float *)xcalloc(n1, sizeof(float));
  int ne[OHMG_MAX];
  int nl = hmg_levels(P->n, ne);
  for (int k = 0; k < nl; ++k) {
    size_t m = (size_t)(ne[k] - 1) * (size_t)(ne[k] - 1);
    w->hr[k] = (double *)xcalloc(m, sizeof(double));
    w->hb[k] = (double *)xcalloc(m, sizeof(double));
    w->hx[k] = (double *)xcalloc(m, sizeof(double));
  }
}

static void work_free(owork *w) {
  free(w->r); free(w->z); free(w->t); free(w->b); free(w->x); free(w->q); free(w->out);
  free(w->r1); free(w->e1);
  free(w->rf); free(w->df); free(w->tf); free(w->zf); free(w->r1f);
  for (int k = 0; k < OHMG_MAX; ++k) {
    free(w->hr[k]);
    free(w->hb[k]);
    free(w->hx[k]);
  }
  memset(w, 0, sizeof(*w));
}

static float *to_float(const double *v, int n) {
  float *f = (float *)xcalloc((size_t)n, sizeof(float));
  for (int i = 0; i < n; ++i) f[i] = (float)v[i];
  return f;
}

/* capmode 0: per-row caps from A's pattern ("fill = nnz of A"); 1: unlimited */
static int pmg_init(opmg *G, const oprob *P, double kappa, double dt, double theta, double tau, int nu1, int nu2,
                    double tol, int maxcyc, int prec, int coarse, int solver, int capmode) {
  memset(G, 0, sizeof(*G));
  G->P = P;
  G->dt = dt;
  G->theta = theta;
  G->nu1 = nu1;
  G->nu2 = nu2;
  G->tol = tol;
  G->maxcyc = maxcyc;
  G->prec = prec;
  G->coarse = coarse;
  G->solver = solver;
  csr_axpby_same(&P->M, theta * kappa * dt, &P->K, &G->A);
  csr_axpby_same(&P->M, -(1.0 - theta) * kappa * dt, &P->K, &G->B);
  if (solver == 1) {
    G->dg = (double *)xcalloc((size_t)G->A.nr, sizeof(double));
    for (int i = 0; i < G->A.nr; ++i)
      for (int k = G->A.rp[i]; k < G->A.rp[i + 1]; ++k)
        if (G->A.ci[k] == i) G->dg[i] = G->A.v[k];
    for (int i = 0; i < G->A.nr; ++i)
      if (!(G->dg[i] > 0.0)) return -4;
    return 0;
  }
  int *lc = (int *)xcalloc((size_t)G->A.nr, sizeof(int)), *uc = (int *)xcalloc((size_t)G->A.nr, sizeof(int));
  if (capmode == 0)
    caps_from_pattern(&G->A, lc, uc);
  else
    for (int i = 0; i < G->A.nr; ++i) lc[i] = uc[i] = G->A.nr;
  int rc = ilut_factor(&G->A, tau, lc, uc, &G->S);
  free(lc);
  free(uc);
  if (rc) return -4;
  /* coarse operator: the same problem rediscretised at p = 1 with the same dt and theta */
  ocsr A1;
  csr_axpby_same(&P->M1, theta * kappa * dt, &P->K1, &A1);
  rc = coarse == 0 ? band_factor(&A1, &G->A1) : hmg_init(&G->H, P->n, &A1);
  csr_free(&A1);
  if (rc) return -4;
  if (prec == 1) {
    G->Af = to_float(G->A.v, G->A.nnz);
    G->Lf = to_float(G->S.L.v, G->S.L.nnz);
    G->Uf = to_float(G->S.U.v, G->S.U.nnz);
    G->Pf = to_float(P->P.v, P->P.nnz);
    G->imlp = (float *)xcalloc((size_t)P->ndof, sizeof(float));
    G->iml1 = (float *)xcalloc((size_t)P->ndof1, sizeof(float));
    for (int i = 0; i < P->ndof; ++i) G->imlp[i] = (float)(1.0 / P->MLp[i]);
    for (int j = 0; j < P->ndof1; ++j) G->iml1[j] = (float)(1.0 / P->ML1[j]);
  }
  return 0;
}

static void pmg_free(opmg *G) {
  csr_free(&G->A);
  csr_free(&G->B);
  ilut_free(&G->S);
  band_free(&G->A1);
  hmg_free(&G->H);
  free(G->dg);
  free(G->Af);
  free(G->Lf);
  free(G->Uf);
  free(G->Pf);
  free(G->imlp);
  free(G->iml1);
  memset(G, 0, sizeof(*G));
}

/* step 3 of the V-cycle: A_{h,1} e_1 = r_1, exactly or by one W-cycle from zero */
static void coarse_solve(const opmg *G, owork *w, const double *r1, double *e1) {
  if (G->coarse == 0) {
    band_solve(&G->A1, r1, e1);
    return;
  }
  for (int j = 0; j < G->P->ndof1; ++j) e1[j] = 0.0;
  hmg_wcycle(&G->H, 0, r1, e1, w->hr, w->hb, w->hx);
}

/* One p-multigrid V-cycle on A x = b (Sec. 4, steps 1-5), FP64. */
static void pmg_vcycle(const opmg *G, owork *w, const double *b, double *x) {
  const oprob *P = G->P;
  int n = P->ndof, n1 = P->ndof1;
  /* 1. nu1 pre-smoothing steps x := x + S (b - A x), eq:smooth */
  for (int m = 0; m < G->nu1; ++m) {
    residual(&G->A, b, x, w->r);
    ilut_apply(&G->S, w->r, w->z);
    for (int i = 0; i < n; ++i) x[i] += w->z[i];
  }
  /* 2. residual restricted to p = 1: r_1 = (M_1^L)^{-1} P_p^1 (b - A x), P_p^1 = (P_1^p)^T */
  residual(&G->A, b, x, w->r);
  csr_mtv(&P->P, w->r, w->r1);
  for (int j = 0; j < n1; ++j) w->r1[j] /= P->ML1[j];
  /* 3. residual equation A_{h,1} e_1 = r_1, eq:res */
  coarse_solve(G, w, w->r1, w->e1);
  /* 4. prolongation and update x := x + (M_p^L)^{-1} P_1^p e_1, eq:prolongation */
  csr_mv(&P->P, w->e1, w->t);
  for (int i = 0; i < n; ++i) x[i] += w->t[i] / P->MLp[i];
  /* 5. nu2 post-smoothing steps */
  for (int m = 0; m < G->nu2; ++m) {
    residual(&G->A, b, x, w->r);
    ilut_apply(&G->S, w->r, w->z);
    for (int i = 0; i < n; ++i) x[i] += w->z[i];
  }
}

/* FP32 building blocks of the refined V-cycle: matrices and vectors in FP32 */
static void residual_f(const ocsr *A, const float *Av, const float *b, const float *x, float *r) {
  for (int i = 0; i < A->nr; ++i) {
    float s = 0.0f;
    for (int k = A->rp[i]; k < A->rp[i + 1]; ++k) s += Av[k] * x[A->ci[k]];
    r[i] = b[i] - s;
  }
}

static void ilut_apply_f(const oilut *F, const float *Lv, const float *Uv, const float *r, float *z) {
  int n = F->n;
  for (int i = 0; i < n; ++i) {
    float s = r[i];
    for (int k = F->L.rp[i]; k < F->L.rp[i + 1]; ++k) s -= Lv[k] * z[F->L.ci[k]];
    z[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    float s = z[i];
    for (int k = F->U.rp[i] + 1; k < F->U.rp[i + 1]; ++k) s -= Uv[k] * z[F->U.ci[k]];
    z[i] = s / Uv[F->U.rp[i]];
  }
}

/* One V-cycle in FP32 on A d = r from d = 0 (correction form), with the p = 1 solve in FP64
 * (step 12 of the method's FP32-refinement variant: the V-cycle is the preconditioner of an FP64
 * refinement loop). */
static void pmg_vcycle_f(const opmg *G, owork *w, const float *r, float *d) {
  const oprob *P = G->P;
  int n = P->ndof, n1 = P->ndof1;
  for (int i = 0; i < n; ++i) d[i] = 0.0f;
  for (int m = 0; m < G->nu1; ++m) {
    residual_f(&G->A, G->Af, r, d, w->tf);
    ilut_apply_f(&G->S, G->Lf, G->Uf, w->tf, w->zf);
    for (int i = 0; i < n; ++i) d[i] += w->zf[i];
  }
  residual_f(&G->A, G->Af, r, d, w->tf);
  for (int j = 0; j < n1; ++j) w->r1f[j] = 0.0f;
  for (int i = 0; i < n; ++i)
    for (int k = P->P.rp[i]; k < P->P.rp[i + 1]; ++k) w->r1f[P->P.ci[k]] += G->Pf[k] * w->tf[i];
  for (int j = 0; j < n1; ++j) w->r1[j] = (double)(w->r1f[j] * G->iml1[j]);
  coarse_solve(G, w, w->r1, w->e1);
  for (int j = 0; j < n1; ++j) w->r1f[j] = (float)w->e1[j];
  for (int i = 0; i < n; ++i) {
    float s = 0.0f;
    for (int k = P->P.rp[i]; k < P->P.rp[i + 1]; ++k) s += G->Pf[k] * w->r1f[P->P.ci[k]];
    d[i] += s * G->imlp[i];
  }
  for (int m = 0; m < G->nu2; ++m) {
    residual_f(&G->A, G->Af, r, d, w->tf);
    ilut_apply_f(&G->S, G->Lf, G->Uf, w->tf, w->zf);
    for (int i = 0; i < n; ++i) d[i] += w->zf[i];
  }
}

/* Conjugate gradients preconditioned by diag(A) (the comparison solver of Sec. 4 and Sec. 5),
 * textbook recursion, from the guess in x until ||r||_2 <= tol ||b||_2 or maxcyc iterations. */
static int pcg_solve(const opmg *G, owork *w, int lvl, const double *b, double *x, double bn) {
  int n = G->A.nr;
  double *r = w->r, *z = w->z, *p = w->t, *q = w->q;
  residual(&G->A, b, x, r);
  double rho_old = 0.0;
  for (int it = 0;; ++it) {
    double rn = nrm2(n, r);
    if (!isfinite(rn)) return -7;
    if (rn <= G->tol * bn) return 0;
    if (it >= G->maxcyc) return -5;
    for (int i = 0; i < n; ++i) z[i] = r[i] / G->dg[i];
    double rho = dot(n, r, z);
    if (it == 0)
      for (int i = 0; i < n; ++i) p[i] = z[i];
    else
      for (int i = 0; i < n; ++i) p[i] = z[i] + (rho / rho_old) * p[i];
    csr_mv(&G->A, p, q);
    double alpha = rho / dot(n, p, q);
    for (int i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    rho_old = rho;
    w->cyc[lvl]++;
  }
}

/* Spatial solve of A x = b from the guess in x until ||b - A x||_2 <= tol ||b||_2 (reading:
 * relative to the right-hand side) or maxcyc cycles / iterations; counters of MGRIT level lvl. */
static int pmg_solve(const opmg *G, owork *w, int lvl, const double *b, double *x) {
  int n = G->P->ndof;
  double bn = nrm2(n, b);
  w->sol[lvl]++;
  if (bn == 0.0) {
    /* a zero right-hand side has the exact solution x = 0 (a relative stop test cannot be met
     * from a non-zero guess) */
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    return 0;
  }
  if (G->solver == 1) return pcg_solve(G, w, lvl, b, x, bn);
  for (int c = 0;; ++c) {
    residual(&G->A, b, x, w->r);
    double rn = nrm2(n, w->r);
    if (!isfinite(rn)) return -7;
    if (rn <= G->tol * bn) return 0;
    if (c >= G->maxcyc) return -5;
    if (G->prec == 0) {
      pmg_vcycle(G, w, b, x);
    } else {
      for (int i = 0; i < n; ++i) w->rf[i] = (float)w->r[i];
      pmg_vcycle_f(G, w, w->rf, w->df);
      for (int i = 0; i < n; ++i) x[i] += (double)w->df[i];
    }
    w->cyc[lvl]++;
  }
}

/* Test entry: solve (M + theta kappa dt K) x = b from guess x with the chosen solver. */
ORC_API int orc_pmg_solve(const oprob *P, double kappa, double dt, double theta, double tau, int nu1, int nu2,
                          double tol, int maxcyc, int prec, int coarse, int solver, int capmode, const double *b,
                          double *x, int *cycles) {
  opmg G;
  owork w;
  work_init(&w, P);
  int rc = pmg_init(&G, P, kappa, dt, theta, tau, nu1, nu2, tol, maxcyc, prec, coarse, solver, capmode);
  if (rc == 0) rc = pmg_solve(&G, &w, 0, b, x);
  *cycles = (int)w.cyc[0];
  pmg_free(&G);
  work_free(&w);
  return rc;
}

/* Test entries of the p = 1 h-multigrid of A_{h,1} = M_1 + theta kappa dt K_1:
 * orc_hmg_info: levels and elements per direction of each (out: ne[OHMG_MAX]);
 * orc_hmg_matrix: shape / CSR of level k's operator (which 0) or prolongation P[k] (which 1);
 * orc_hmg_cycles: ncyc W-cycles on A_{h,1} x = b from the x given;
 * orc_gs_sweep: one four-colour Gauss-Seidel sweep (dir +1 / -1) on A_{h,1} x = b. */
ORC_API int orc_hmg_info(const oprob *P, int *ne) { return hmg_levels(P->n, ne); }

ORC_API int orc_hmg_matrix(const oprob *P, double kappa, double dt, double theta, int k, int which, int *shape3,
                           int *rp, int *ci, double *v) {
  ocsr A1;
  ohmg H;
  csr_axpby_same(&P->M1, theta * kappa * dt, &P->K1, &A1);
  int rc = hmg_init(&H, P->n, &A1);
  csr_free(&A1);
  if (rc == 0 && (k < 0 || k >= H.nlev || (which == 1 && k == 0))) rc = -1;
  if (rc == 0) {
    const ocsr *a = which == 0 ? &H.A[k] : &H.P[k];
    shape3[0] = a->nr;
    shape3[1] = a->nc;
    shape3[2] = a->nnz;
    if (rp) {
      memcpy(rp, a->rp, sizeof(int) * (size_t)(a->nr + 1));
      memcpy(ci, a->ci, sizeof(int) * (size_t)a->nnz);
      memcpy(v, a->v, sizeof(double) * (size_t)a->nnz);
    }
  }
  hmg_free(&H);
  return rc;
}

ORC_API int orc_hmg_cycles(const oprob *P, double kappa, double dt, double theta, int ncyc, const double *b,
                           double *x) {
  ocsr A1;
  ohmg H;
  owork w;
  work_init(&w, P);
  csr_axpby_same(&P->M1, theta * kappa * dt, &P->K1, &A1);
  int rc = hmg_init(&H, P->n, &A1);
  csr_free(&A1);
  for (int c = 0; rc == 0 && c < ncyc; ++c) hmg_wcycle(&H, 0, b, x, w.hr, w.hb, w.hx);
  hmg_free(&H);
  work_free(&w);
  return rc;
}

ORC_API void orc_gs_sweep(const oprob *P, double kappa, double dt, double theta, int dir, const double *b,
                          double *x) {
  ocsr A1;
  csr_axpby_same(&P->M1, theta * kappa * dt, &P->K1, &A1);
  gs_sweep(&A1, P->n - 1, b, x, dir);
  csr_free(&A1);
}

/* ------------------------------------------------------------------ */
/* Time stepping (Sec. 2, eq:los; Sec. 3, eq:mgrit)                     */
/* ------------------------------------------------------------------ */

/* source time factor: kind 0 -> 1, kind 1 -> exp(-t) */
static double tfac(int kind, double t) { return kind == 1 ? exp(-t) : 1.0; }

/* source weight of the theta-scheme step k -> k+1 with step dt: dt (theta s(t_{k+1}) +
 * (1 - theta) s(t_k)) (reading: the source is weighted like the diffusion term; eq:los has a
 * time-independent f, where this is dt f) */
static double src_weight(int kind, double theta, double dt, int k) {
  return dt * (theta * tfac(kind, (k + 1) * dt) + (1.0 - theta) * tfac(kind, k * dt));
}

/* Sequential theta-scheme with direct solves:
 *   U_0 = u0;  (M + theta kappa dt K) U_{k+1} = (M - (1 - theta) kappa dt K) U_k + w_k F,
 * k = 0..Nt-1, w_k = src_weight (eq:los), i.e. the block forward solve of A u = g in eq:mgrit.
 * U is (Nt+1) x ndof, row-major. */
ORC_API int orc_sequential_theta(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind,
                                 double theta, const double *u0, double *U) {
  int n = P->ndof;
  double dt = T / Nt;
  ocsr A, B;
  csr_axpby_same(&P->M, theta * kappa * dt, &P->K, &A);
  csr_axpby_same(&P->M, -(1.0 - theta) * kappa * dt, &P->K, &B);
  oband f;
  int rc = band_factor(&A, &f);
  csr_free(&A);
  if (rc) {
    csr_free(&B);
    return -4;
  }
  double *rhs = (double *)xcalloc((size_t)n, sizeof(double));
  memcpy(U, u0, sizeof(double) * (size_t)n);
  for (int k = 0; k < Nt; ++k) {
    csr_mv(&B, U + (size_t)k * n, rhs);
    double c = src_weight(tkind, theta, dt, k);
    for (int i = 0; i < n; ++i) rhs[i] += c * F[i];
    band_solve(&f, rhs, U + (size_t)(k + 1) * n);
  }
  free(rhs);
  csr_free(&B);
  band_free(&f);
  return 0;
}

/* implicit Euler (theta = 1) */
ORC_API int orc_sequential(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind,
                           const double *u0, double *U) {
  return orc_sequential_theta(P, kappa, T, Nt, F, tkind, 1.0, u0, U);
}

/* Sequential theta-scheme with the iterative spatial solver (guess: previous step). */
ORC_API int orc_sequential_pmg(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind,
                               double theta, const double *u0, double tau, double stol, int maxcyc, int prec,
                               int coarse, int solver, double *U, long long *cycles) {
  int n = P->ndof;
  double dt = T / Nt;
  opmg G;
  owork w;
  work_init(&w, P);
  int rc = pmg_init(&G, P, kappa, dt, theta, tau, 1, 1, stol, maxcyc, prec, coarse, solver, 0);
  memcpy(U, u0, sizeof(double) * (size_t)n);
  for (int k = 0; k < Nt && rc == 0; ++k) {
    csr_mv(&G.B, U + (size_t)k * n, w.b);
    double c = src_weight(tkind, theta, dt, k);
    for (int i = 0; i < n; ++i) w.b[i] += c * F[i];
    memcpy(U + (size_t)(k + 1) * n, U + (size_t)k * n, sizeof(double) * (size_t)n);
    rc = pmg_solve(&G, &w, 0, w.b, U + (size_t)(k + 1) * n);
  }
  *cycles = w.cyc[0];
  pmg_free(&G);
  work_free(&w);
  return rc;
}

/* ------------------------------------------------------------------ */
/* MGRIT (Sec. 3)                                                      */
/* ------------------------------------------------------------------ */

/* Level l of the time hierarchy: N_l intervals of size dt_l = m^l dt (rediscretised,
 * Sec. 3), the vector v (u at level 0, the correction at coarser levels) and the
 * right-hand side g of A^{(l)} v = g^{(l)} at coarse levels.  The step of A^{(l)} is
 *   level 0:  v_{k+1} = Psi_0 (B_0 v_k + w_k F)      (one spatial solve)
 *   level l:  v_{k+1} = Psi_l B_l v_k + g_{k+1}       (Psi_l = A_l^{-1})
 * with A_l, B_l the theta-scheme operators of dt_l, and the residual of A^{(l)} v = g at point k
 * is step(v_{k-1}) - v_k. */
typedef struct {
  int Nl;
  double dt;
  opmg G;
  double *v, *g;
} olev;

typedef struct {
  const oprob *P;
  double kappa, T, theta;
  int Nt, m, nlev, guess, cycle, nth;
  const double *F;
  int tkind;
  olev *L;
  owork *W; /* one per thread */
  int rc;
} omgrit;

#ifdef _OPENMP
#include <omp.h>
static int thread_id(void) { return omp_get_thread_num(); }
#else
static int thread_id(void) { return 0; }
#endif

/* one step at level l from v[k] to target k+1, written into out (which may alias v[k+1]).
 * guess policy: 0 zero, 1 previous point, 2 current value of the target at level 0 (it carries
 * the previous MGRIT iterate) and the previous point at coarser levels (whose state restarts
 * from zero in every cycle, so their targets carry no information in the first sweeps). */
static void mg_step(omgrit *S, owork *w, int l, int k, double *out) {
  olev *L = &S->L[l];
  int n = S->P->ndof;
  const double *vk = L->v + (size_t)k * n;
  csr_mv(&L->G.B, vk, w->b);
  if (l == 0) {
    double c = src_weight(S->tkind, S->theta, L->dt, k);
    for (int i = 0; i < n; ++i) w->b[i] += c * S->F[i];
  }
  const double *tgt = L->v + (size_t)(k + 1) * n;
  const double *gk = l > 0 ? L->g + (size_t)(k + 1) * n : NULL; /* coarse right-hand side, added after the solve */
  for (int i = 0; i < n; ++i) {
    if (S->guess == 0)
      w->x[i] = 0.0;
    else if (S->guess == 1 || l > 0)
      w->x[i] = vk[i];
    else
      w->x[i] = tgt[i];
  }
  int rc = pmg_solve(&L->G, w, l, w->b, w->x);
  if (rc) {
#ifdef _OPENMP
#pragma omp critical(orc_rc)
#endif
    if (!S->rc) S->rc = rc;
  }
  for (int i = 0; i < n; ++i) out[i] = w->x[i] + (gk ? gk[i] : 0.0);
}

/* F-relaxation: inside every coarse interval propagate from its C-point to its F-points
 * (intervals are independent: one thread each) */
static void f_relax(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof, m = S->m, nint = (L->Nl + m - 1) / m;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(S->nth)
#endif
  for (int j = 0; j < nint; ++j) {
    owork *w = &S->W[thread_id()];
    for (int s = 1; s < m && j * m + s <= L->Nl; ++s) {
      int k = j * m + s - 1;
      mg_step(S, w, l, k, L->v + (size_t)(k + 1) * n);
    }
  }
}

/* C-relaxation: every C-point j m (j >= 1) from its preceding F-point. */
static void c_relax(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof, m = S->m, nc = L->Nl / m;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(S->nth)
#endif
  for (int j = 1; j <= nc; ++j) mg_step(S, &S->W[thread_id()], l, j * m - 1, L->v + (size_t)(j * m) * n);
}

/* residual at the C-points after relaxation, r_j = step(v_{jm-1}) - v_{jm}, injected as the
 * right-hand side of level l+1 (its point j).  Returns sum_j ||r_j||^2 (summed in j order). */
static double c_residual_inject(omgrit *S, int l) {
  olev *L = &S->L[l], *C = &S->L[l + 1];
  int n = S->P->ndof, m = S->m, nc = L->Nl / m;
  memset(C->g, 0, sizeof(double) * (size_t)n); /* point 0 is exact: zero residual */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(S->nth)
#endif
  for (int j = 1; j <= nc; ++j) {
    owork *w = &S->W[thread_id()];
    mg_step(S, w, l, j * m - 1, w->out);
    double *gj = C->g + (size_t)j * n;
    const double *vj = L->v + (size_t)(j * m) * n;
    for (int i = 0; i < n; ++i) gj[i] = w->out[i] - vj[i];
  }
  double s2 = 0.0;
  for (int j = 1; j <= nc; ++j) {
    const double *gj = C->g + (size_t)j * n;
    for (int i = 0; i < n; ++i) s2 += gj[i] * gj[i];
  }
  return s2;
}

/* coarsest level: block forward solve of A^{(L)} v = g (sequential time stepping) */
static void coarsest_solve(omgrit *S, int l) {
  olev *L = &S->L[l];
  int n = S->P->ndof;
  memcpy(L->v, L->g, sizeof(double) * (size_t)n);
  for (int k = 0; k < L->Nl; ++k) mg_step(S, &S->W[0], l, k, L->v + (size_t)(k + 1) * n);
}

static void level_solve(omgrit *S, int l, int kind);

/* One MGRIT cycle on level l >= 1 for A^{(l)} v = g^{(l)} from the current v (Sec. 3, the MGRIT
 * recursion): FCF-relaxation, the C-point residual injected into level l + 1, the level-(l+1)
 * correction from zero, v := v + P v^{(l+1)} by ideal interpolation (correct the C-points, then
 * F-relax from them). */
static void mgrit_cycle(omgrit *S, int l, int kind) {
  olev *L = &S->L[l], *C = &S->L[l + 1];
  int n = S->P->ndof, m = S->m;
  f_relax(S, l);
  c_relax(S, l);
  f_relax(S, l);
  (void)c_residual_inject(S, l);
  memset(C->v, 0, sizeof(double) * (size_t)(C->Nl + 1) * n);
  level_solve(S, l + 1, kind);
  for (int j = 1; j * m <= L->Nl; ++j) {
    double *vj = L->v + (size_t)(j * m) * n;
    const double *ej = C->v + (size_t)j * n;
    for (int i = 0; i < n; ++i) vj[i] += ej[i];
  }
  f_relax(S, l);
}

/* Approximate solve of the level-l problem from its current v (Sec. 3, cycle types): the coarsest
 * level by its block forward solve; otherwise one cycle (kind 0, V-cycle), two cycles (kind 1,
 * W-cycle), or one F-cycle followed by one V-cycle (kind 2, F-cycle). */
static void level_solve(omgrit *S, int l, int kind) {
  if (l == S->nlev - 1) {
    coarsest_solve(S, l);
    return;
  }
  if (kind == 0) {
    mgrit_cycle(S, l, 0);
  } else if (kind == 1) {
    mgrit_cycle(S, l, 1);
    mgrit_cycle(S, l, 1);
  } else {
    mgrit_cycle(S, l, 2);
    mgrit_cycle(S, l, 0);
  }
}

/* MGRIT on level 0 for the theta-scheme.  Hierarchy: N_l = N_t / m^l, coarsening stops at level
 * max_levels-1 or when N_l <= coarsest_max.  Initial guess: U_0 = u0, U_k = 0 for k >= 1
 * (reading).  Iteration: FCF-relaxation and the level-0 C-point residual; stop when
 * ||r^{(k)}|| <= tol ||r^{(0)}|| (reading of the relative residual criterion of Sec. 5); else the
 * level-1 correction by level_solve and the C-point update.  The converged iterate is the
 * post-FCF state, whose F-points are already consistent.
 * iopt = {m, max_levels, coarsest_max, max_iter, maxcyc, guess, cycle (0 V, 1 W, 2 F), prec,
 *         coarse, solver, nthreads};
 * dopt = {tol, tau, stol, ctol, theta}: spatial solves stop at stol on level 0 and at ctol on the
 * coarse levels (ctol <= 0: stol).  The paper fixes neither; the coarse levels only supply
 * corrections, so their tolerance changes the convergence rate, not the fixed point that the
 * level-0 test measures.
 * out: iters, V-cycles (or CG iterations), spatial solves; res_hist (up to 200 entries). */
ORC_API int orc_mgrit(const oprob *P, double kappa, double T, int Nt, const double *F, int tkind, const double *u0,
                      const int *iopt, const double *dopt, double *U, int *iters, long long *cycles,
                      long long *solves, double *res_hist) {
  int m = iopt[0], max_levels = iopt[1], coarsest_max = iopt[2], max_iter = iopt[3], maxcyc = iopt[4];
  double tol = dopt[0], tau = dopt[1], stol = dopt[2], ctol = dopt[3];
  int n = P->ndof;
  omgrit S;
  memset(&S, 0, sizeof(S));
  S.P = P;
  S.kappa = kappa;
  S.T = T;
  S.theta = dopt[4];
  S.Nt = Nt;
  S.m = m;
  S.F = F;
  S.tkind = tkind;
  S.guess = iopt[5];
  S.cycle = iopt[6];
  S.nth = iopt[10] < 1 ? 1 : iopt[10];
  int nlev = 1;
  {
    int Nl = Nt;
    while (nlev < max_levels && nlev < OMAXLEV && Nl > coarsest_max && Nl / m >= 1) {
      Nl /= m;
      ++nlev;
    }
  }
  S.nlev = nlev;
  S.L = (olev *)xcalloc((size_t)nlev, sizeof(olev));
  S.W = (owork *)xcalloc((size_t)S.nth, sizeof(owork));
  for (int t = 0; t < S.nth; ++t) work_init(&S.W[t], P);
  int Nl = Nt;
  double dt = T / Nt;
  int rc = 0;
  for (int l = 0; l < nlev; ++l) {
    S.L[l].Nl = Nl;
    S.L[l].dt = dt;
    if (rc == 0)
      rc = pmg_init(&S.L[l].G, P, kappa, dt, S.theta, tau, 1, 1, (l > 0 && ctol > 0) ? ctol : stol, maxcyc, iopt[7],
                    iopt[8], iopt[9], 0);
    S.L[l].v = l == 0 ? U : (double *)xcalloc((size_t)(Nl + 1) * n, sizeof(double));
    S.L[l].g = l == 0 ? NULL : (double *)xcalloc((size_t)(Nl + 1) * n, sizeof(double));
    Nl /= m;
    dt *= m;
  }
  int it = 0;
  if (rc == 0) {
    memset(U, 0, sizeof(double) * (size_t)(Nt + 1) * n);
    memcpy(U, u0, sizeof(double) * (size_t)n);
    if (nlev == 1) {
      /* no coarsening possible: sequential solve at level 0 */
      for (int k = 0; k < Nt; ++k) mg_step(&S, &S.W[0], 0, k, U + (size_t)(k + 1) * n);
    } else {
      double r0 = -1.0;
      for (;;) {
        f_relax(&S, 0);
        c_relax(&S, 0);
        f_relax(&S, 0);
        double rn = sqrt(c_residual_inject(&S, 0));
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
        level_solve(&S, 1, S.cycle);
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
  for (int t = 0; t < S.nth; ++t)
    for (int l = 0; l < nlev; ++l) {
      cyc += S.W[t].cyc[l];
      sol += S.W[t].sol[l];
    }
  for (int l = 0; l < nlev; ++l) {
    pmg_free(&S.L[l].G);
    if (l > 0) {
      free(S.L[l].v);
      free(S.L[l].g);
    }
  }
  for (int t = 0; t < S.nth; ++t) work_free(&S.W[t]);
  *iters = it;
  *cycles = cyc;
  *solves = sol;
  free(S.L);
  free(S.W);
  return rc;
}
