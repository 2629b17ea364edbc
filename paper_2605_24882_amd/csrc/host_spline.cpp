// Host-side construction of the spline space tables used by the device kernels:
// Gauss-Legendre rules, B-spline values/derivatives on the dyadic knot vectors,
// the knot-insertion (prolongation) matrix between consecutive levels, and the
// interface gluing of the six cube-sphere patches.
//
// Sec. 2.1 (p-open knot vectors, B-spline recursion), Sec. 2.3 (dyadic knot
// vectors Xi_{j,p}, the continuous space S^0_{j,p}), Sec. 3.2 (quadrature of the
// pulled-back forms; the rule is Gauss-Legendre with p+1 points per direction).
#include "gf_internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <tuple>

namespace gf {

// q-point Gauss-Legendre rule on [0,1]: Newton iteration on the three-term
// Legendre recurrence, started from the Chebyshev-like guess cos(pi (i-1/4)/(q+1/2)).
void gauss_legendre(int q, std::vector<double> &x, std::vector<double> &w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = z; p0 = 1.0; }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = z; p0 = 1.0; }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    // map [-1,1] -> [0,1], ascending order
    x[q - 1 - i] = 0.5 * (z + 1.0);
    w[q - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) scaled by 1/2
  }
}

// Knot k of the p-open dyadic knot vector with nel elements, in units of 1/nel.
static inline int knot_int(int k, int p, int nel) {
  int v = k - p;
  return v < 0 ? 0 : (v > nel ? nel : v);
}

// Values and first derivatives of the p+1 B-splines that are non-zero on element e
// (indices e..e+p) at the local abscissa u in [0,1] of that element.  The recursion
// raises the degree one step at a time on the knots around the element; a term with
// a vanishing knot difference is dropped.
void element_basis(int p, int nel, int e, double u, double *val, double *der) {
  const double x = (e + u) / nel;
  auto kn = [&](int k) { return (double)knot_int(k, p, nel) / nel; };
  // basis functions of degree d non-zero on span [kn(e+p), kn(e+p+1)): indices e+p-d .. e+p
  // N[d][r] holds function index e+p-d+r
  double N[8][8] = {{0}};
  N[0][0] = 1.0;
  for (int d = 1; d <= p; ++d) {
    for (int r = 0; r <= d; ++r) {
      int l = e + p - d + r;  // global index at degree d
      double v = 0.0;
      // left term: (x - xi_l)/(xi_{l+d} - xi_l) * b_l^{d-1}; b_l^{d-1} = N[d-1][r-1]
      if (r - 1 >= 0) {
        double den = kn(l + d) - kn(l);
        if (den > 0.0) v += (x - kn(l)) / den * N[d - 1][r - 1];
      }
      // right term: (xi_{l+d+1} - x)/(xi_{l+d+1} - xi_{l+1}) * b_{l+1}^{d-1}; = N[d-1][r]
      if (r <= d - 1) {
        double den = kn(l + d + 1) - kn(l + 1);
        if (den > 0.0) v += (kn(l + d + 1) - x) / den * N[d - 1][r];
      }
      N[d][r] = v;
    }
  }
  for (int r = 0; r <= p; ++r) val[r] = N[p][r];
  if (p == 0) {
    der[0] = 0.0;
    return;
  }
  // derivative: p/(xi_{l+p}-xi_l) b_l^{p-1} - p/(xi_{l+p+1}-xi_{l+1}) b_{l+1}^{p-1}
  for (int r = 0; r <= p; ++r) {
    int l = e + r;
    double dv = 0.0;
    if (r - 1 >= 0) {
      double den = kn(l + p) - kn(l);
      if (den > 0.0) dv += p / den * N[p - 1][r - 1];
    }
    if (r <= p - 1) {
      double den = kn(l + p + 1) - kn(l + 1);
      if (den > 0.0) dv -= p / den * N[p - 1][r];
    }
    der[r] = dv;
  }
}

// Knot-insertion matrix from level lc to lc+1 (dense, row-major (n1f x n1c)), built by
// inserting the midpoints of all coarse spans one at a time (Boehm's algorithm).  Each
// row holds one control point of the refined representation as a combination of the
// coarse control points.
std::vector<double> refinement_matrix(int p, int lc) {
  int nel = 1 << lc;
  std::vector<double> U;  // current knot vector in units of 1/(2 nel)
  for (int k = 0; k < nel + 2 * p + 1; ++k) U.push_back(2.0 * knot_int(k, p, nel));
  int nc = nel + p;
  // rows: current control points, each a combination of nc coarse points
  std::vector<std::vector<double>> Q(nc, std::vector<double>(nc, 0.0));
  for (int i = 0; i < nc; ++i) Q[i][i] = 1.0;
  for (int e = 0; e < nel; ++e) {
    double ubar = 2.0 * e + 1.0;  // midpoint of coarse span e
    // span index k with U[k] <= ubar < U[k+1]
    int k = -1;
    for (int i = 0; i + 1 < (int)U.size(); ++i)
      if (U[i] <= ubar && ubar < U[i + 1]) { k = i; break; }
    if (k < 0) throw std::runtime_error("knot insertion: span not found");
    int n = (int)Q.size();
    std::vector<std::vector<double>> R(n + 1, std::vector<double>(nc, 0.0));
    for (int i = 0; i <= n; ++i) {
      if (i <= k - p) {
        R[i] = Q[i];
      } else if (i >= k + 1) {
        R[i] = Q[i - 1];
      } else {
        double a = (ubar - U[i]) / (U[i + p] - U[i]);
        for (int c = 0; c < nc; ++c) R[i][c] = a * Q[i][c] + (1.0 - a) * Q[i - 1][c];
      }
    }
    Q.swap(R);
    U.insert(U.begin() + k + 1, ubar);
  }
  int nf = (int)Q.size();
  if (nf != 2 * nel + p) throw std::runtime_error("knot insertion: wrong fine size");
  std::vector<double> P((size_t)nf * nc);
  for (int i = 0; i < nf; ++i)
    for (int c = 0; c < nc; ++c) P[(size_t)i * nc + c] = Q[i][c];
  return P;
}

// Cube-face placement of the six patches: v = (coords) with a = 2s-1, b = 2t-1.
//   0: ( 1, a, b)  1: (-1, b, a)  2: ( b, 1, a)  3: ( a,-1, b)  4: ( a, b, 1)  5: ( b, a,-1)
// fixed_axis/fixed_sign give the constant coordinate, a_axis/b_axis where a and b go.
const PatchFrame kPatchFrames[6] = {
    {0, +1, 1, 2}, {0, -1, 2, 1}, {1, +1, 2, 0}, {1, -1, 0, 2}, {2, +1, 0, 1}, {2, -1, 1, 0}};

// Interface gluing on one level: local (m, iy, ix) -> global id.  Each coefficient is
// attached to the cube-surface point of its Greville abscissae, which has integer
// coordinates in units of 1/(p nel); equal points on different faces are the same
// unknown.  Numbering: patches 0..5, then iy, then ix, next id to every new point.
void glue_patches(int p, int lev, std::vector<int> &l2g, int &N) {
  int nel = 1 << lev, n1 = nel + p;
  std::vector<int> G(n1);  // p*nel*greville(i)
  for (int i = 0; i < n1; ++i) {
    int s = 0;
    for (int k = 1; k <= p; ++k) s += knot_int(i + k, p, nel);
    G[i] = (p == 0) ? 0 : s;
  }
  const int span = p * nel;
  std::map<std::tuple<int, int, int>, int> seen;
  l2g.assign((size_t)6 * n1 * n1, -1);
  N = 0;
  for (int m = 0; m < 6; ++m) {
    const PatchFrame &f = kPatchFrames[m];
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        int c[3];
        c[f.fixed_axis] = f.fixed_sign * span;
        c[f.a_axis] = 2 * G[ix] - span;
        c[f.b_axis] = 2 * G[iy] - span;
        auto key = std::make_tuple(c[0], c[1], c[2]);
        auto it = seen.find(key);
        int g;
        if (it == seen.end()) {
          g = N++;
          seen.emplace(key, g);
        } else {
          g = it->second;
        }
        l2g[((size_t)m * n1 + iy) * n1 + ix] = g;
      }
  }
}

// Interfaces of NURBS patches (Sec. 2.2: neighbouring patch maps agree on the shared edge up to the
// orientation of the reference square).  Edge e of patch m: 0 is t = 0, 1 is t = 1, 2 is s = 0,
// 3 is s = 1.  Two edges are the same curve with the same parametrisation (or its reverse) when
// their rows of control points and weights agree point by point (relative tolerance 1e-12 of the
// surface's extent) and their knot vectors agree (or are mirrored); such edges are glued, and the
// coefficients along them identified in the same or the reverse order.  Corners join through the
// edges (union-find), so any number of patches may meet at a point.  Numbering as glue_patches:
// patches in order, then iy, then ix, the next id to every new class.
namespace {
struct EdgeData {
  std::vector<double> pts;  // [k][4]
  std::vector<double> knots;
};

EdgeData nurbs_edge(const NurbsHost &g, int m, int e) {
  const int *pi = &g.pinfo[5 * (size_t)m];
  const int ns = pi[0], nt = pi[1];
  const double *U = &g.knots[pi[2]], *V = &g.knots[pi[3]], *C = &g.ctrl[4 * (size_t)pi[4]];
  EdgeData d;
  const bool along_s = (e < 2);
  const int n = along_s ? ns : nt;
  for (int k = 0; k < n; ++k) {
    const int a = along_s ? k : (e == 2 ? 0 : ns - 1);
    const int b = along_s ? (e == 0 ? 0 : nt - 1) : k;
    const double *c = C + 4 * ((size_t)b * ns + a);
    d.pts.insert(d.pts.end(), c, c + 4);
  }
  if (along_s) d.knots.assign(U, U + ns + g.du + 1);
  else d.knots.assign(V, V + nt + g.dv + 1);
  return d;
}

// 0: different curves, 1: same orientation, 2: reversed
int edges_match(const EdgeData &x, const EdgeData &y, double tol) {
  if (x.pts.size() != y.pts.size() || x.knots.size() != y.knots.size()) return 0;
  const size_t n = x.pts.size() / 4, nk = x.knots.size();
  for (int rev = 0; rev < 2; ++rev) {
    bool ok = true;
    for (size_t k = 0; k < n && ok; ++k) {
      const double *a = &x.pts[4 * k], *b = &y.pts[4 * (rev ? n - 1 - k : k)];
      for (int c = 0; c < 3; ++c) ok = ok && std::fabs(a[c] - b[c]) <= tol;
      ok = ok && std::fabs(a[3] - b[3]) <= 1e-12 * std::max(std::fabs(a[3]), std::fabs(b[3]));
    }
    for (size_t k = 0; k < nk && ok; ++k) {
      const double u = x.knots[k], v = rev ? 1.0 - y.knots[nk - 1 - k] : y.knots[k];
      ok = std::fabs(u - v) <= 1e-14;
    }
    if (ok) return rev ? 2 : 1;
  }
  return 0;
}

int uf_find(std::vector<int> &par, int i) {
  while (par[i] != i) {
    par[i] = par[par[i]];
    i = par[i];
  }
  return i;
}
}  // namespace

void glue_patches_nurbs(const NurbsHost &g, int p, int lev, std::vector<int> &l2g, int &N) {
  const int np = g.npatch, n1 = (1 << lev) + p;
  double ext = 0.0;
  for (size_t i = 0; i < g.ctrl.size(); i += 4)
    for (int c = 0; c < 3; ++c) ext = std::max(ext, std::fabs(g.ctrl[i + c]));
  const double tol = 1e-12 * std::max(ext, 1e-300);
  std::vector<EdgeData> edges;
  for (int m = 0; m < np; ++m)
    for (int e = 0; e < 4; ++e) {
      edges.push_back(nurbs_edge(g, m, e));
      // an edge collapsed to a point (a pole) has a singular metric: not supported
      const auto &pts = edges.back().pts;
      bool point = true;
      for (size_t k = 4; k < pts.size() && point; k += 4)
        for (int c = 0; c < 3; ++c) point = point && std::fabs(pts[k + c] - pts[c]) <= tol;
      if (point) fail(GF_EUNSUPPORTED, "a patch edge collapses to a point (degenerate patch)");
    }
  auto coef = [&](int m, int e, int i) -> int {
    const int iy = e == 0 ? 0 : e == 1 ? n1 - 1 : i;
    const int ix = e == 2 ? 0 : e == 3 ? n1 - 1 : i;
    return (m * n1 + iy) * n1 + ix;
  };
  std::vector<int> par((size_t)np * n1 * n1);
  for (size_t i = 0; i < par.size(); ++i) par[i] = (int)i;
  std::vector<int> partners(edges.size(), 0);
  for (size_t a = 0; a < edges.size(); ++a)
    for (size_t b = a + 1; b < edges.size(); ++b) {
      const int how = edges_match(edges[a], edges[b], tol);
      if (!how) continue;
      if (++partners[a] > 1 || ++partners[b] > 1) fail(GF_EINVAL, "a patch edge is shared by more than two patches");
      const int ma = (int)a / 4, ea = (int)a % 4, mb = (int)b / 4, eb = (int)b % 4;
      for (int i = 0; i < n1; ++i) {
        const int x = uf_find(par, coef(ma, ea, i)), y = uf_find(par, coef(mb, eb, how == 2 ? n1 - 1 - i : i));
        if (x != y) par[std::max(x, y)] = std::min(x, y);
      }
    }
  l2g.assign(par.size(), -1);
  std::vector<int> id(par.size(), -1);
  N = 0;
  for (size_t i = 0; i < par.size(); ++i) {
    const int r = uf_find(par, (int)i);
    if (id[r] < 0) id[r] = N++;
    l2g[i] = id[r];
  }
}

// ------------------------------------------------------------------ NURBS evaluation on the host
namespace {
// knot span of u among the n basis functions of degree d (u = 1 in the last non-empty span)
int host_span(const double *U, int n, int d, double u) {
  if (u >= U[n]) {
    int i = n - 1;
    while (i > d && U[i] >= U[i + 1]) --i;
    return i;
  }
  int lo = d, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (u < U[mid]) hi = mid;
    else lo = mid;
  }
  return lo;
}

// values and first derivatives of the d+1 non-zero basis functions span-d .. span at u
void host_basis(const double *U, int span, int d, double u, double *N, double *dN) {
  double tri[5][5];
  tri[0][0] = 1.0;
  for (int k = 1; k <= d; ++k)
    for (int j = 0; j <= k; ++j) {
      const int i = span - k + j;
      double v = 0.0;
      if (j > 0 && U[i + k] > U[i]) v += (u - U[i]) / (U[i + k] - U[i]) * tri[k - 1][j - 1];
      if (j < k && U[i + k + 1] > U[i + 1]) v += (U[i + k + 1] - u) / (U[i + k + 1] - U[i + 1]) * tri[k - 1][j];
      tri[k][j] = v;
    }
  for (int j = 0; j <= d; ++j) {
    N[j] = tri[d][j];
    const int i = span - d + j;
    double v = 0.0;
    if (d > 0) {
      if (j > 0 && U[i + d] > U[i]) v += d * tri[d - 1][j - 1] / (U[i + d] - U[i]);
      if (j < d && U[i + d + 1] > U[i + 1]) v -= d * tri[d - 1][j] / (U[i + d + 1] - U[i + 1]);
    }
    dN[j] = v;
  }
}
}  // namespace

void nurbs_eval(const NurbsHost &g, int m, double s, double t, double X[3], double Xs[3], double Xt[3]) {
  const int *pi = &g.pinfo[5 * (size_t)m];
  const int ns = pi[0], nt = pi[1];
  const double *U = &g.knots[pi[2]], *V = &g.knots[pi[3]], *C = &g.ctrl[4 * (size_t)pi[4]];
  const int su = host_span(U, ns, g.du, s), sv = host_span(V, nt, g.dv, t);
  double Nu[5], dNu[5], Nv[5], dNv[5];
  host_basis(U, su, g.du, s, Nu, dNu);
  host_basis(V, sv, g.dv, t, Nv, dNv);
  double P[4] = {0, 0, 0, 0}, Ps[4] = {0, 0, 0, 0}, Pt[4] = {0, 0, 0, 0};
  for (int b = 0; b <= g.dv; ++b)
    for (int a = 0; a <= g.du; ++a) {
      const double *c = C + 4 * ((size_t)(sv - g.dv + b) * ns + (su - g.du + a));
      const double h[4] = {c[0] * c[3], c[1] * c[3], c[2] * c[3], c[3]};
      for (int k = 0; k < 4; ++k) {
        P[k] += Nu[a] * Nv[b] * h[k];
        Ps[k] += dNu[a] * Nv[b] * h[k];
        Pt[k] += Nu[a] * dNv[b] * h[k];
      }
    }
  for (int k = 0; k < 3; ++k) {
    X[k] = P[k] / P[3];
    Xs[k] = (Ps[k] - X[k] * Ps[3]) / P[3];
    Xt[k] = (Pt[k] - X[k] * Pt[3]) / P[3];
  }
}

// Closest point on the NURBS surface: every patch is sampled on a grid of parameters, the patches
// whose best sample lies within twice the best distance (plus a margin) are refined by Gauss-Newton
// steps on |F_m(s, t) - P|^2 with (s, t) kept in [0, 1]^2, and the closest result wins (the lower
// patch index on ties, as on shared edges).
void nurbs_locate(const NurbsHost &g, const double P[3], int *patch, double *s_out, double *t_out, double *dist) {
  constexpr int G = 17;
  std::vector<double> best(g.npatch, 1e300), bs(g.npatch), bt(g.npatch);
  double X[3], Xs[3], Xt[3];
  for (int m = 0; m < g.npatch; ++m)
    for (int a = 0; a < G; ++a)
      for (int b = 0; b < G; ++b) {
        const double s = a / (G - 1.0), t = b / (G - 1.0);
        nurbs_eval(g, m, s, t, X, Xs, Xt);
        const double d2 = (X[0] - P[0]) * (X[0] - P[0]) + (X[1] - P[1]) * (X[1] - P[1]) + (X[2] - P[2]) * (X[2] - P[2]);
        if (d2 < best[m]) {
          best[m] = d2;
          bs[m] = s;
          bt[m] = t;
        }
      }
  const double gbest = *std::min_element(best.begin(), best.end());
  double win = 1e300;
  *patch = -1;
  for (int m = 0; m < g.npatch; ++m) {
    if (std::sqrt(best[m]) > 2.0 * std::sqrt(gbest) + 1e-3 * (1.0 + std::sqrt(gbest))) continue;
    double s = bs[m], t = bt[m];
    for (int it = 0; it < 60; ++it) {
      nurbs_eval(g, m, s, t, X, Xs, Xt);
      const double r[3] = {X[0] - P[0], X[1] - P[1], X[2] - P[2]};
      const double a11 = Xs[0] * Xs[0] + Xs[1] * Xs[1] + Xs[2] * Xs[2];
      const double a12 = Xs[0] * Xt[0] + Xs[1] * Xt[1] + Xs[2] * Xt[2];
      const double a22 = Xt[0] * Xt[0] + Xt[1] * Xt[1] + Xt[2] * Xt[2];
      const double g1 = Xs[0] * r[0] + Xs[1] * r[1] + Xs[2] * r[2];
      const double g2 = Xt[0] * r[0] + Xt[1] * r[1] + Xt[2] * r[2];
      const double det = a11 * a22 - a12 * a12;
      if (!(det > 0.0)) break;
      const double ds = -(a22 * g1 - a12 * g2) / det, dt = -(a11 * g2 - a12 * g1) / det;
      const double sn = std::min(1.0, std::max(0.0, s + ds)), tn = std::min(1.0, std::max(0.0, t + dt));
      const double step = std::fabs(sn - s) + std::fabs(tn - t);
      s = sn;
      t = tn;
      if (step < 1e-15) break;
    }
    nurbs_eval(g, m, s, t, X, Xs, Xt);
    const double d2 = (X[0] - P[0]) * (X[0] - P[0]) + (X[1] - P[1]) * (X[1] - P[1]) + (X[2] - P[2]) * (X[2] - P[2]);
    if (d2 < win * (1.0 - 1e-12) - 1e-300) {
      win = d2;
      *patch = m;
      *s_out = s;
      *t_out = t;
    }
  }
  *dist = std::sqrt(win);
}

// Jacobi elliptic functions by the arithmetic-geometric mean and the descending recurrence of the
// amplitude (Abramowitz & Stegun, Sec. 16.4): with a_0 = 1, b_0 = sqrt(1-q), c_0 = sqrt(q),
// a_n = (a_{n-1}+b_{n-1})/2, b_n = sqrt(a_{n-1} b_{n-1}), c_n = (a_{n-1}-b_{n-1})/2 until c_N is
// negligible, phi_N = 2^N a_N u and phi_{n-1} = (phi_n + asin(c_n sin(phi_n)/a_n))/2; then
// sn = sin(phi_0), cn = cos(phi_0), dn = cos(phi_0)/cos(phi_1 - phi_0).  K(q) = pi/(2 a_N).
namespace {
int agm(double q, double *a, double *c) {
  a[0] = 1.0;
  double b = std::sqrt(1.0 - q);
  c[0] = std::sqrt(q);
  int n = 0;
  while (n < 30 && std::fabs(c[n]) > 1e-17 * a[n]) {
    a[n + 1] = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    ++n;
  }
  return n;
}
}  // namespace

void jacobi_sncndn(double u, double q, double *sn, double *cn, double *dn) {
  double a[32], c[32];
  const int n = agm(q, a, c);
  double phi = std::ldexp(a[n] * u, n);
  double prev = phi;
  for (int k = n; k >= 1; --k) {
    prev = phi;
    phi = 0.5 * (phi + std::asin(c[k] * std::sin(phi) / a[k]));
  }
  *sn = std::sin(phi);
  *cn = std::cos(phi);
  *dn = (n == 0) ? 1.0 : *cn / std::cos(prev - phi);
}

double complete_k(double q) {
  double a[32], c[32];
  const int n = agm(q, a, c);
  return M_PI / (2.0 * a[n]);
}

}  // namespace gf
