// host_setup.cpp -- see host_setup.hpp.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <queue>
#include <stdexcept>

namespace pmg {

// ---------------------------------------------------------------------------------------
// dense symmetric eigen-solver: cyclic Jacobi (textbook, e.g. Golub & Van Loan Sec. 8.5)
// ---------------------------------------------------------------------------------------
void sym_eig(const Dense& A0, std::vector<double>& lam, Dense& Z) {
  const int n = A0.r;
  Dense A = A0;
  Z = Dense(n, n);
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  double fro = 0.0;
  for (double v : A.a) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
    if (std::sqrt(off) <= 1e-17 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (apq == 0.0) continue;
        double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          double zkp = Z(k, p), zkq = Z(k, q);
          Z(k, p) = c * zkp - s * zkq;
          Z(k, q) = s * zkp + c * zkq;
        }
      }
  }
  lam.assign(n, 0.0);
  for (int i = 0; i < n; ++i) lam[i] = A(i, i);
}

// Golub-Welsch: nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// Legendre recurrence, weights 2 * (first eigenvector component)^2, then mapped to [0,1].
void gauss01(int q, std::vector<double>& x, std::vector<double>& w) {
  Dense J(q, q);
  for (int k = 1; k < q; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    J(k - 1, k) = J(k, k - 1) = b;
  }
  std::vector<double> lam;
  Dense Z;
  sym_eig(J, lam, Z);
  std::vector<int> ord(q);
  for (int i = 0; i < q; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    int e = ord[i];
    x[i] = 0.5 * (lam[e] + 1.0);
    w[i] = Z(0, e) * Z(0, e);  // 2 * z0^2 on [-1,1], halved on [0,1]
  }
  // symmetrise (the rule is symmetric about 1/2) to remove eigen-solver noise
  for (int i = 0; i < q / 2; ++i) {
    double xm = 0.5 * (x[i] + (1.0 - x[q - 1 - i])), wm = 0.5 * (w[i] + w[q - 1 - i]);
    x[i] = xm;
    x[q - 1 - i] = 1.0 - xm;
    w[i] = w[q - 1 - i] = wm;
  }
  if (q % 2 == 1) x[q / 2] = 0.5;
}

// ---------------------------------------------------------------------------------------
// B-splines: triangular evaluation of the non-zero functions of one knot span
// ---------------------------------------------------------------------------------------
static void span_values(const std::vector<double>& U, int span, double x, int deg, double* N) {
  // N[a] = phi_{span-deg+a, deg}(x), built up degree by degree from phi_{span,0} = 1
  double left[64], right[64];
  N[0] = 1.0;
  for (int j = 1; j <= deg; ++j) {
    left[j] = x - U[span + 1 - j];
    right[j] = U[span + j] - x;
    double carry = 0.0;
    for (int r = 0; r < j; ++r) {
      double den = right[r + 1] + left[j - r];
      double tmp = den != 0.0 ? N[r] / den : 0.0;
      N[r] = carry + right[r + 1] * tmp;
      carry = left[j - r] * tmp;
    }
    N[j] = carry;
  }
}

void bspline_values(const std::vector<double>& U, int p, int span, double x, double* val, double* der) {
  span_values(U, span, x, p, val);
  if (!der) return;
  if (p == 0) {
    der[0] = 0.0;
    return;
  }
  double low[64];
  span_values(U, span, x, p - 1, low);  // low[a] = phi_{span-p+1+a, p-1}
  for (int a = 0; a <= p; ++a) {
    int i = span - p + a;
    double d = 0.0;
    if (a >= 1) {
      double den = U[i + p] - U[i];
      if (den != 0.0) d += p * low[a - 1] / den;
    }
    if (a <= p - 1) {
      double den = U[i + p + 1] - U[i + 1];
      if (den != 0.0) d -= p * low[a] / den;
    }
    der[a] = d;
  }
}

static std::vector<double> open_knots(int n, int p) {
  std::vector<double> U;
  for (int i = 0; i < p; ++i) U.push_back(0.0);
  for (int i = 0; i <= n; ++i) U.push_back((double)i / n);
  for (int i = 0; i < p; ++i) U.push_back(1.0);
  return U;
}

// weights of the separable parametrisations (see header)
static double weight(int kind, double s) {
  if (kind == 0) return 1.0;
  if (kind == 1) return 1.0 + s;
  if (kind == 2) return 1.0 / (1.0 + s);
  // rational quadratic quarter circle c(t) = N(t) / D(t), middle weight sqrt(2)/2
  const double w = std::sqrt(0.5);
  double t = s, u = 1.0 - t;
  double Nx = u * u + 2.0 * t * u * w, Ny = 2.0 * t * u * w + t * t;
  double D = u * u + 2.0 * t * u * w + t * t;
  double dNx = -2.0 * u + 2.0 * w * (1.0 - 2.0 * t), dNy = 2.0 * w * (1.0 - 2.0 * t) + 2.0 * t;
  double dD = -2.0 * u + 2.0 * w * (1.0 - 2.0 * t) + 2.0 * t;
  double cx = (dNx * D - Nx * dD) / (D * D), cy = (dNy * D - Ny * dD) / (D * D);
  double speed = std::sqrt(cx * cx + cy * cy);
  return kind == 3 ? speed : 1.0 / speed;
}

Dense weighted_1d(int n, int pa, int pb, int da, int db, int wkind, int q) {
  std::vector<double> Ua = open_knots(n, pa), Ub = open_knots(n, pb), gx, gw;
  gauss01(q, gx, gw);
  Dense W(n + pa, n + pb);
  const double h = 1.0 / n;
  double va[64], dva[64], vb[64], dvb[64];
  for (int e = 0; e < n; ++e)
    for (int g = 0; g < q; ++g) {
      double s = (e + gx[g]) * h;
      double wt = gw[g] * h * weight(wkind, s);
      bspline_values(Ua, pa, e + pa, s, va, dva);
      bspline_values(Ub, pb, e + pb, s, vb, dvb);
      for (int a = 0; a <= pa; ++a) {
        double fa = da ? dva[a] : va[a];
        for (int b = 0; b <= pb; ++b) {
          double fb = db ? dvb[b] : vb[b];
          W(e + a, e + b) += fa * fb * wt;
        }
      }
    }
  return W;
}

std::vector<double> mode_load_1d(int n, int p, int k, int wkind, int q) {
  std::vector<double> U = open_knots(n, p), gx, gw;
  gauss01(q, gx, gw);
  std::vector<double> out(n + p, 0.0);
  const double h = 1.0 / n;
  double v[64];
  for (int e = 0; e < n; ++e)
    for (int g = 0; g < q; ++g) {
      double s = (e + gx[g]) * h;
      double f = k == 0 ? 1.0 : std::sin(k * M_PI * s);
      bspline_values(U, p, e + p, s, v, nullptr);
      for (int a = 0; a <= p; ++a) out[e + a] += v[a] * f * gw[g] * h * weight(wkind, s);
    }
  return out;
}

Csr kron_interior(int Ny, int Nx, int My, int Mx, int bylo, int byhi, int bxlo, int bxhi,
                  const std::vector<KronTerm>& terms) {
  Csr A;
  const int ry = Ny - 2, rx = Nx - 2, cy = My - 2, cx = Mx - 2;
  A.nr = ry * rx;
  A.nc = cy * cx;
  A.rp.assign(A.nr + 1, 0);
  for (int iy = 1; iy <= ry; ++iy)
    for (int ix = 1; ix <= rx; ++ix) {
      int row = (iy - 1) * rx + (ix - 1);
      for (int jy = std::max(1, iy + bylo); jy <= std::min(My - 2, iy + byhi); ++jy)
        for (int jx = std::max(1, ix + bxlo); jx <= std::min(Mx - 2, ix + bxhi); ++jx) {
          double v = 0.0;
          for (const KronTerm& t : terms) v += t.c * (*t.Y)(iy, jy) * (*t.X)(ix, jx);
          A.ci.push_back((jy - 1) * cx + (jx - 1));
          A.v.push_back(v);
        }
      A.rp[row + 1] = (int)A.ci.size();
    }
  return A;
}

// ---------------------------------------------------------------------------------------
// ILUT (Saad's dual-threshold incomplete LU): elimination order from a min-heap of the
// pending lower columns of the work row.
// ---------------------------------------------------------------------------------------
bool ilut(const Csr& A, double tau, const std::vector<int>& lcap, const std::vector<int>& ucap, Csr& L, Csr& U,
          std::string& err) {
  const int n = A.nr;
  std::vector<double> w(n, 0.0);
  std::vector<char> in(n, 0);
  std::vector<int> touched;
  touched.reserve(4096);
  L = Csr();
  U = Csr();
  L.nr = L.nc = U.nr = U.nc = n;
  L.rp.assign(n + 1, 0);
  U.rp.assign(n + 1, 0);
  std::vector<int> udiag(n, 0);  // position of u_ii in U
  struct Cand {
    int j;
    double a;
  };
  std::vector<Cand> lo, up;
  for (int i = 0; i < n; ++i) {
    std::priority_queue<int, std::vector<int>, std::greater<int>> pend;
    double nrm = 0.0;
    for (int t = A.rp[i]; t < A.rp[i + 1]; ++t) {
      int j = A.ci[t];
      w[j] = A.v[t];
      in[j] = 1;
      touched.push_back(j);
      if (j < i) pend.push(j);
      nrm += A.v[t] * A.v[t];
    }
    const double thr = tau * std::sqrt(nrm);
    while (!pend.empty()) {
      int k = pend.top();
      pend.pop();
      if (w[k] == 0.0) continue;
      double lk = w[k] / U.v[udiag[k]];
      if (std::fabs(lk) < thr) {
        w[k] = 0.0;
        continue;
      }
      w[k] = lk;
      for (int t = udiag[k] + 1; t < U.rp[k + 1]; ++t) {
        int j = U.ci[t];
        if (!in[j]) {
          in[j] = 1;
          w[j] = 0.0;
          touched.push_back(j);
          if (j < i) pend.push(j);
        }
        w[j] -= lk * U.v[t];
      }
    }
    lo.clear();
    up.clear();
    for (int j : touched) {
      double a = w[j];
      if (j == i || a == 0.0 || std::fabs(a) < thr) continue;
      (j < i ? lo : up).push_back({j, a});
    }
    auto bigger = [](const Cand& x, const Cand& y) {
      double ax = std::fabs(x.a), ay = std::fabs(y.a);
      return ax != ay ? ax > ay : x.j < y.j;
    };
    auto bycol = [](const Cand& x, const Cand& y) { return x.j < y.j; };
    if ((int)lo.size() > lcap[i]) {
      std::sort(lo.begin(), lo.end(), bigger);
      lo.resize(lcap[i]);
    }
    if ((int)up.size() > ucap[i]) {
      std::sort(up.begin(), up.end(), bigger);
      up.resize(ucap[i]);
    }
    std::sort(lo.begin(), lo.end(), bycol);
    std::sort(up.begin(), up.end(), bycol);
    for (const Cand& c : lo) {
      L.ci.push_back(c.j);
      L.v.push_back(c.a);
    }
    double piv = in[i] ? w[i] : 0.0;
    udiag[i] = (int)U.ci.size();
    U.ci.push_back(i);
    U.v.push_back(piv);
    for (const Cand& c : up) {
      U.ci.push_back(c.j);
      U.v.push_back(c.a);
    }
    L.rp[i + 1] = (int)L.ci.size();
    U.rp[i + 1] = (int)U.ci.size();
    for (int j : touched) {
      w[j] = 0.0;
      in[j] = 0;
    }
    touched.clear();
    if (!(piv > 0.0) || !std::isfinite(piv)) {
      err = "ILUT: non-positive pivot at row " + std::to_string(i);
      return false;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------------------
// blocked level schedule
// ---------------------------------------------------------------------------------------
TriSchedule build_schedule(const Csr& T, bool upper, int bs, int cap) {
  TriSchedule S;
  const int n = T.nr;
  S.n = n;
  S.upper = upper;
  S.bs = bs = std::max(1, std::min(bs, n));
  const int nb = (n + bs - 1) / bs;
  S.nblocks = nb;
  auto blk = [bs](int i) { return i / bs; };
  // block levels from off-block dependencies
  std::vector<int> lev(nb, 0);
  auto dep_level = [&](int b) {
    int l = 0;
    int r0 = b * bs, r1 = std::min(n, r0 + bs);
    for (int i = r0; i < r1; ++i)
      for (int t = T.rp[i]; t < T.rp[i + 1]; ++t) {
        int j = T.ci[t], bj = blk(j);
        if (bj != b) l = std::max(l, lev[bj] + 1);
      }
    return l;
  };
  // blocks in dependency order, each at the first level after its dependencies that still has
  // room for its rows (cap rows per level, 0: no cap); a block's arithmetic does not depend on
  // its level, only the number of levels does
  std::vector<int> used;
  auto place = [&](int b) {
    const int m = std::min(n, b * bs + bs) - b * bs;
    int l = dep_level(b);
    while (cap > 0 && l < (int)used.size() && used[l] + m > cap) ++l;
    if (l >= (int)used.size()) used.resize(l + 1, 0);
    used[l] += m;
    lev[b] = l;
  };
  if (!upper)
    for (int b = 0; b < nb; ++b) place(b);
  else
    for (int b = nb - 1; b >= 0; --b) place(b);
  int nlev = 0;
  for (int b = 0; b < nb; ++b) nlev = std::max(nlev, lev[b] + 1);
  S.nlev = nlev;
  std::vector<std::vector<int>> byl(nlev);
  for (int b = 0; b < nb; ++b) byl[lev[b]].push_back(b);
  S.lev_ptr.assign(nlev + 1, 0);
  S.orp.push_back(0);
  for (int l = 0; l < nlev; ++l) {
    int lstart = (int)S.row.size();
    for (int b : byl[l]) {
      int r0 = b * bs, r1 = std::min(n, r0 + bs), m = r1 - r0;
      int qb = (int)S.row.size() - lstart;  // block start within the level
      // dense diagonal block and its inverse (forward/back substitution on unit vectors)
      Dense D(m, m), X(m, m);
      for (int a = 0; a < m; ++a) {
        int i = r0 + a;
        if (!upper) D(a, a) = 1.0;
        for (int t = T.rp[i]; t < T.rp[i + 1]; ++t) {
          int j = T.ci[t];
          if (blk(j) == b) D(a, j - r0) = T.v[t];
        }
      }
      if (!upper) {
        for (int c = 0; c < m; ++c) {
          X(c, c) = 1.0;
          for (int r = c + 1; r < m; ++r) {
            double s = 0.0;
            for (int k = c; k < r; ++k) s += D(r, k) * X(k, c);
            X(r, c) = -s;
          }
        }
      } else {
        for (int c = m - 1; c >= 0; --c) {
          X(c, c) = 1.0 / D(c, c);
          for (int r = c - 1; r >= 0; --r) {
            double s = 0.0;
            for (int k = r + 1; k <= c; ++k) s += D(r, k) * X(k, c);
            X(r, c) = -s / D(r, r);
          }
        }
      }
      for (int a = 0; a < m; ++a) {
        int i = r0 + a;
        S.row.push_back(i);
        for (int t = T.rp[i]; t < T.rp[i + 1]; ++t) {
          int j = T.ci[t];
          if (blk(j) != b) {
            S.oci.push_back(j);
            S.ov.push_back(T.v[t]);
          }
        }
        S.orp.push_back((int)S.oci.size());
        S.doff.push_back((int64_t)S.dval.size());
        if (!upper) {
          S.dq0.push_back(qb);
          S.dcnt.push_back(a + 1);
          for (int c = 0; c <= a; ++c) S.dval.push_back(X(a, c));
        } else {
          S.dq0.push_back(qb + a);
          S.dcnt.push_back(m - a);
          for (int c = a; c < m; ++c) S.dval.push_back(X(a, c));
        }
      }
    }
    S.lev_ptr[l + 1] = (int)S.row.size();
    S.max_rows = std::max(S.max_rows, S.lev_ptr[l + 1] - S.lev_ptr[l]);
  }
  return S;
}

}  // namespace pmg
