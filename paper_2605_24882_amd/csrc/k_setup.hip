// Setup kernels: metric terms at the Gauss points, the matrix-free sum-factorised
// operator application, stencil extraction by probing, diagonals, the element-wise
// white-noise load and the coarse-level Cholesky factors.
#include "gf_internal.h"

namespace gf {

// cube-face frames of the six patches (same table as the host's kPatchFrames)
__constant__ int c_frames[6][4] = {{0, 1, 1, 2}, {0, -1, 2, 1}, {1, 1, 2, 0},
                                   {1, -1, 0, 2}, {2, 1, 0, 1}, {2, -1, 1, 0}};

// Surface point and its parameter derivatives for patch m at (s, t) (Sec. 2.2 maps).
// xh = v/|v| has d xh = (dv - xh (xh . dv))/|v|; the perturbed surface r(xh) xh with
// r = 1 + amp sin(3x) sin(2y) cos(z) has d(r xh) = (grad r . d xh) xh + r d xh.
__device__ void surface_derivs(int m, double s, double t, double amp, double Fs[3], double Ft[3]) {
  const int fa = c_frames[m][0], fs = c_frames[m][1], aa = c_frames[m][2], ba = c_frames[m][3];
  double v[3], vs[3] = {0, 0, 0}, vt[3] = {0, 0, 0};
  v[fa] = (double)fs;
  v[aa] = 2.0 * s - 1.0;
  v[ba] = 2.0 * t - 1.0;
  vs[aa] = 2.0;
  vt[ba] = 2.0;
  const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double xh[3], xs[3], xt[3];
  for (int i = 0; i < 3; ++i) xh[i] = v[i] / nv;
  const double ps = xh[0] * vs[0] + xh[1] * vs[1] + xh[2] * vs[2];
  const double pt = xh[0] * vt[0] + xh[1] * vt[1] + xh[2] * vt[2];
  for (int i = 0; i < 3; ++i) {
    xs[i] = (vs[i] - xh[i] * ps) / nv;
    xt[i] = (vt[i] - xh[i] * pt) / nv;
  }
  if (amp == 0.0) {
    for (int i = 0; i < 3; ++i) { Fs[i] = xs[i]; Ft[i] = xt[i]; }
    return;
  }
  const double X = xh[0], Y = xh[1], Z = xh[2];
  const double r = 1.0 + amp * sin(3.0 * X) * sin(2.0 * Y) * cos(Z);
  const double gr[3] = {3.0 * amp * cos(3.0 * X) * sin(2.0 * Y) * cos(Z),
                        2.0 * amp * sin(3.0 * X) * cos(2.0 * Y) * cos(Z), -amp * sin(3.0 * X) * sin(2.0 * Y) * sin(Z)};
  const double rs = gr[0] * xs[0] + gr[1] * xs[1] + gr[2] * xs[2];
  const double rt = gr[0] * xt[0] + gr[1] * xt[1] + gr[2] * xt[2];
  for (int i = 0; i < 3; ++i) {
    Fs[i] = rs * xh[i] + r * xs[i];
    Ft[i] = rt * xh[i] + r * xt[i];
  }
}

// ---- rational tensor-product B-spline patches (Sec. 2.2: the patch maps of a NURBS surface)
constexpr int kMaxGeomDeg = 4;

// knot span i with U[i] <= u < U[i+1] among the n basis functions of degree d (open knot vector
// U[0 .. n+d]); u = U[n] falls into the last non-empty span
__device__ int nurbs_span(const double *U, int n, int d, double u) {
  if (u >= U[n]) {
    int i = n - 1;
    while (i > d && U[i] >= U[i + 1]) --i;
    return i;
  }
  int lo = d, hi = n;  // U[lo] <= u < U[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (u < U[mid]) hi = mid;
    else lo = mid;
  }
  return lo;
}

// values N[j] and first derivatives dN[j] of the d+1 basis functions span-d+j (j = 0..d) at u, by
// the Cox-de Boor recursion over the degrees 0..d (terms with a vanishing denominator dropped)
__device__ void nurbs_basis(const double *U, int span, int d, double u, double *N, double *dN) {
  double tri[kMaxGeomDeg + 1][kMaxGeomDeg + 1];
  tri[0][0] = 1.0;
  for (int k = 1; k <= d; ++k)
    for (int j = 0; j <= k; ++j) {
      const int i = span - k + j;
      double v = 0.0;
      if (j > 0) {
        const double den = U[i + k] - U[i];
        if (den > 0.0) v += (u - U[i]) / den * tri[k - 1][j - 1];
      }
      if (j < k) {
        const double den = U[i + k + 1] - U[i + 1];
        if (den > 0.0) v += (U[i + k + 1] - u) / den * tri[k - 1][j];
      }
      tri[k][j] = v;
    }
  for (int j = 0; j <= d; ++j) {
    N[j] = tri[d][j];
    const int i = span - d + j;
    double v = 0.0;
    if (d > 0) {
      if (j > 0) {
        const double den = U[i + d] - U[i];
        if (den > 0.0) v += d * tri[d - 1][j - 1] / den;
      }
      if (j < d) {
        const double den = U[i + d + 1] - U[i + 1];
        if (den > 0.0) v -= d * tri[d - 1][j] / den;
      }
    }
    dN[j] = v;
  }
}

// F = P / w with P = sum N_a(s) N_b(t) w_ab X_ab, w = sum N_a N_b w_ab; dF = (dP - F dw) / w
__device__ void nurbs_derivs(const SurfaceArgs &g, int m, double s, double t, double Fs[3], double Ft[3]) {
  const int *pi = g.pinfo + 5 * m;
  const int ns = pi[0], nt = pi[1];
  const double *U = g.knots + pi[2], *V = g.knots + pi[3], *C = g.ctrl + 4 * (int64_t)pi[4];
  const int su = nurbs_span(U, ns, g.du, s), sv = nurbs_span(V, nt, g.dv, t);
  double Nu[kMaxGeomDeg + 1], dNu[kMaxGeomDeg + 1], Nv[kMaxGeomDeg + 1], dNv[kMaxGeomDeg + 1];
  nurbs_basis(U, su, g.du, s, Nu, dNu);
  nurbs_basis(V, sv, g.dv, t, Nv, dNv);
  double P[4] = {0, 0, 0, 0}, Ps[4] = {0, 0, 0, 0}, Pt[4] = {0, 0, 0, 0};  // homogeneous (x w, y w, z w, w)
  for (int b = 0; b <= g.dv; ++b)
    for (int a = 0; a <= g.du; ++a) {
      const double *c = C + 4 * ((int64_t)(sv - g.dv + b) * ns + (su - g.du + a));
      const double h[4] = {c[0] * c[3], c[1] * c[3], c[2] * c[3], c[3]};
      for (int k = 0; k < 4; ++k) {
        P[k] += Nu[a] * Nv[b] * h[k];
        Ps[k] += dNu[a] * Nv[b] * h[k];
        Pt[k] += Nu[a] * dNv[b] * h[k];
      }
    }
  for (int k = 0; k < 3; ++k) {
    const double F = P[k] / P[3];
    Fs[k] = (Ps[k] - F * Ps[3]) / P[3];
    Ft[k] = (Pt[k] - F * Pt[3]) / P[3];
  }
}

// m = w a, G = w a K^-1 at every Gauss point (Sec. 3.2: K first fundamental form,
// a = sqrt(det K)); w is the tensor Gauss weight of the element (area 1/nel^2).
__global__ void k_metric(double *metric, int nel, int q, SurfaceArgs g, const double *gx, const double *gw) {
  const int64_t total = (int64_t)g.npatch * nel * nel * q * q;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  int64_t t = id;
  const int qx = t % q; t /= q;
  const int qy = t % q; t /= q;
  const int ex = t % nel; t /= nel;
  const int ey = t % nel; t /= nel;
  const int m = (int)t;
  const double s = (ex + gx[qx]) / nel, tt = (ey + gx[qy]) / nel;
  double Fs[3], Ft[3];
  if (g.kind == SURF_NURBS) nurbs_derivs(g, m, s, tt, Fs, Ft);
  else surface_derivs(m, s, tt, g.amp, Fs, Ft);
  const double k11 = Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2];
  const double k12 = Fs[0] * Ft[0] + Fs[1] * Ft[1] + Fs[2] * Ft[2];
  const double k22 = Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2];
  const double det = k11 * k22 - k12 * k12;
  const double a = sqrt(det);
  const double w = gw[qx] * gw[qy] / ((double)nel * nel);
  double *o = metric + id * 4;
  o[0] = w * a;
  o[1] = w * a * k22 / det;
  o[2] = -w * a * k12 / det;
  o[3] = w * a * k11 / det;
}

void launch_metric(const Level &L, const SurfaceArgs &g, const double *gx, const double *gw, hipStream_t s) {
  const int64_t total = (int64_t)g.npatch * L.nel * L.nel * L.q * L.q;
  hipLaunchKernelGGL(k_metric, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, L.metric.p, L.nel, L.q, g,
                     gx, gw);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ matrix-free apply
// y = (ca M + cb S) x per column, patch by patch (no interface sum), evaluating the element integrals of
// eq. mass / eq. stiffness at the Q x Q Gauss points on the fly (sum factorisation).  Per element
// (NB = p+1 basis functions per direction, coefficients c[b][a], b along t, a along s):
//   U0[b][qx] = sum_a c[b][a] Bx[qx][a],  U1[b][qx] = sum_a c[b][a] Dx[qx][a]
//   u = sum_b U0 By, us = sum_b U1 By, ut = sum_b U0 Dy                        (at each qy, qx)
//   v = ca m u,  gs = cb (G11 us + G12 ut),  gt = cb (G12 us + G22 ut)
//   V0[b][qx] = sum_qy v By + gt Dy,  V1[b][qx] = sum_qy gs By
//   y_e[b][a] = sum_qx V0 Bx + V1 Dx
// (evaluated one quadrature column qx at a time: only NB-long intermediates are live)
// Every element is evaluated once.  Element rows are coloured by ey mod NB: the rows of one colour
// touch disjoint coefficient rows (ey .. ey+p), so one launch per colour adds them into y (zeroed
// first) without atomics, in a fixed order.  A block runs one element row of one patch for four column
// tiles (one wavefront each, lane = column): the four share each element's metric terms and basis
// tables Bx, Dx, staged in LDS a chunk of elements at a time (the row's By, Dy are uniform loads).  Along the row a wavefront keeps the NB x NB
// coefficients of the current element and an NB-column ring of output sums in registers; column ex
// is complete once element ex is done and is added to y.
constexpr int kSfChunk = 16;  // elements staged per LDS chunk

template <typename T, int P, int Q>
__global__ __launch_bounds__(256) void k_sumfact(const T *__restrict__ metric, const T *__restrict__ basis,
                                                 const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ ca,
                                                 const T *__restrict__ cb, int nel, int n1, int W, int ldb, int ntiles,
                                                 const int *__restrict__ active, int colour, int nrow, int np) {
  constexpr int NB = P + 1, QQ = Q * Q, BT = Q * NB;  // BT: one basis table (Q points x NB functions)
  constexpr int CHUNK = kSfChunk;
  __shared__ T sm[CHUNK][QQ * 4];       // metric terms of the chunk's elements
  __shared__ T sb[CHUNK][2 * BT];       // Bx, Dx of the chunk's elements
  const int ntg = (ntiles + 3) / 4;
  const int tg = blockIdx.x % ntg, rr = (blockIdx.x / ntg) % nrow, m = blockIdx.x / (ntg * nrow);
  if (m >= np) return;
  const int ey = colour + rr * NB;
  if (ey >= nel) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ct = tg * 4 + wave;
  const bool on = ct < ntiles && (!active || active[ct]);
  const int64_t col = (int64_t)ct * CT + lane;
  // the row's basis tables By, Dy are the same for every element of the row: uniform loads (scalar
  // registers); the metric terms and Bx, Dx change per element and are staged in LDS
  const T *By = basis + (size_t)ey * 2 * BT, *Dy = By + BT;
  const T sig = on ? ca[col] : T(0), ss = on ? cb[col] : T(0);
  const int64_t prow = (int64_t)m * W * W;
  // coefficient rows ey .. ey+p of the patch (padded rows ey+P .. ey+2P, columns shifted by P)
  auto xat = [&](int b, int a) { return x[(prow + (int64_t)(ey + b + P) * W + (a + P)) * ldb + col]; };
  auto yadd = [&](int b, int a, T v) {
    T *py = y + (prow + (int64_t)(ey + b + P) * W + (a + P)) * ldb + col;
    *py += v;
  };
  T c[NB][NB], ring[NB][NB];  // ring[b][k]: output column (ex + k) mod NB of coefficient row ey + b
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int k = 0; k < NB; ++k) ring[b][k] = T(0);
  if (on) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int a = 0; a < P; ++a) c[b][a + 1] = xat(b, a);  // columns 0 .. P-1, shifted in below
  }
  for (int e0 = 0; e0 < nel; e0 += CHUNK) {
    const int ne = min(CHUNK, nel - e0);
    __syncthreads();  // the previous chunk's reads are done
    for (int k = threadIdx.x; k < ne * QQ * 4; k += 256)
      sm[k / (QQ * 4)][k % (QQ * 4)] = metric[((((size_t)m * nel + ey) * nel + e0) * QQ) * 4 + k];
    for (int k = threadIdx.x; k < ne * 2 * BT; k += 256)
      sb[k / (2 * BT)][k % (2 * BT)] = basis[(size_t)e0 * 2 * BT + k];
    __syncthreads();
    if (!on) continue;
    for (int el = 0; el < ne; ++el) {
      const int ex = e0 + el;
      // the element's coefficient window: shift by one column, load column ex + P
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int a = 0; a < P; ++a) c[b][a] = c[b][a + 1];
        c[b][P] = xat(b, ex + P);
      }
      const T *Bx = sb[el], *Dx = sb[el] + BT, *mt = sm[el];
      // one quadrature column qx at a time (only NB-long intermediates live); local column a of the
      // element is output column ex + a, ring slot a
#pragma unroll 1
      for (int qx = 0; qx < Q; ++qx) {
        T U0[NB], U1[NB], V0[NB], V1[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          T s0 = 0, s1 = 0;
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            s0 = fma(c[b][a], Bx[qx * NB + a], s0);
            s1 = fma(c[b][a], Dx[qx * NB + a], s1);
          }
          U0[b] = s0;
          U1[b] = s1;
          V0[b] = 0;
          V1[b] = 0;
        }
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
          T u = 0, us = 0, ut = 0;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            u = fma(U0[b], By[qy * NB + b], u);
            us = fma(U1[b], By[qy * NB + b], us);
            ut = fma(U0[b], Dy[qy * NB + b], ut);
          }
          const T *gq = mt + (qy * Q + qx) * 4;
          const T v = sig * gq[0] * u;
          const T gs = ss * (gq[1] * us + gq[2] * ut);
          const T gt = ss * (gq[2] * us + gq[3] * ut);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            V0[b] = fma(v, By[qy * NB + b], fma(gt, Dy[qy * NB + b], V0[b]));
            V1[b] = fma(gs, By[qy * NB + b], V1[b]);
          }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int a = 0; a < NB; ++a)
            ring[b][a] = fma(V0[b], Bx[qx * NB + a], fma(V1[b], Dx[qx * NB + a], ring[b][a]));
      }
      // output column ex is complete: add it to y and rotate the ring by one column
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        yadd(b, ex, ring[b][0]);
#pragma unroll
        for (int k = 0; k < P; ++k) ring[b][k] = ring[b][k + 1];
        ring[b][P] = T(0);
      }
    }
  }
  if (on) {
    // the row's last P output columns nel .. nel+P-1
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int k = 0; k < P; ++k) yadd(b, nel + k, ring[b][k]);
  }
}

// y = 0 on the rows of the patches, active column tiles
template <typename T>
__global__ void k_zero_rows(T *y, int64_t R, int ldb, int ntiles, const int *active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * ldb) return;
  const int ct = (int)(i % ldb) / CT;
  if (active && !active[ct]) return;
  y[i] = T(0);
}

template <typename T>
static const T *metric_of(const Level &L);
template <>
const double *metric_of<double>(const Level &L) { return L.metric.p; }
template <>
const float *metric_of<float>(const Level &L) { return L.metric32.p; }
template <typename T>
static const T *basis_of(const Level &L);
template <>
const double *basis_of<double>(const Level &L) { return L.basis.p; }
template <>
const float *basis_of<float>(const Level &L) { return L.basis32.p; }

template <typename T>
void launch_sumfact_apply(const Level &L, const T *x, T *y, const T *ca, const T *cb, int ldb, int ntiles,
                          const int *active, hipStream_t s) {
  const T *mt = metric_of<T>(L), *bs = basis_of<T>(L);
  if (L.q != L.p + 1 && L.q != L.p + 2) fail(GF_EUNSUPPORTED, "quadrature order out of range");
  const bool q2 = L.q == L.p + 2;
  const int64_t tot = L.R * ldb;
  hipLaunchKernelGGL(k_zero_rows<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, y, L.R, ldb, ntiles,
                     active);
  const int NB = L.p + 1, ntg = (ntiles + 3) / 4;
  for (int colour = 0; colour < NB && colour < L.nel; ++colour) {
    const int nrow = (L.nel - colour + NB - 1) / NB;
    const dim3 grid((unsigned)(L.npatch * nrow * ntg)), block(256);
    switch (L.p) {
#define GF_SF(PP)                                                                                              \
  case PP:                                                                                                     \
    if (q2)                                                                                                    \
      hipLaunchKernelGGL((k_sumfact<T, PP, PP + 2>), grid, block, 0, s, mt, bs, x, y, ca, cb, L.nel, L.n1, L.W, \
                         ldb, ntiles, active, colour, nrow, L.npatch);                                         \
    else                                                                                                       \
      hipLaunchKernelGGL((k_sumfact<T, PP, PP + 1>), grid, block, 0, s, mt, bs, x, y, ca, cb, L.nel, L.n1, L.W, \
                         ldb, ntiles, active, colour, nrow, L.npatch);                                         \
    break;
      GF_SF(1) GF_SF(2) GF_SF(3) GF_SF(4) GF_SF(5)
#undef GF_SF
      default: fail(GF_EUNSUPPORTED, "degree out of range");
    }
  }
  HIPCHK(hipGetLastError());
}
template void launch_sumfact_apply<double>(const Level &, const double *, double *, const double *, const double *,
                                           int, int, const int *, hipStream_t);
template void launch_sumfact_apply<float>(const Level &, const float *, float *, const float *, const float *, int,
                                          int, const int *, hipStream_t);

// ------------------------------------------------------------------ stencil by probing
// Column c < S*S probes colour c = (iy mod S)*S + (ix mod S) for M, column S*S + c the same
// colour for S.  Within the (2p+1)^2 window of any coefficient each colour occurs exactly
// once, so (A x_c)[row] is the single stencil entry of that colour.
__global__ void k_probe(double *x, int ldb, int n1, int W, int P, int Sw, int64_t R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= R) return;
  const int lx = (int)(r % W) - P, ly = (int)((r / W) % W) - P;
  const bool inside = lx >= 0 && lx < n1 && ly >= 0 && ly < n1;
  const int colour = inside ? (ly % Sw) * Sw + (lx % Sw) : -1;
  for (int c = threadIdx.x; c < ldb; c += blockDim.x) {
    const double v = (inside && c < 2 * Sw * Sw && c % (Sw * Sw) == colour) ? 1.0 : 0.0;
    x[r * ldb + c] = v;
  }
}

void launch_probe_vectors(const Level &L, double *x, int ldb, hipStream_t s) {
  dim3 block(64, 4);
  dim3 grid((unsigned)((L.R + block.y - 1) / block.y));
  hipLaunchKernelGGL(k_probe, grid, block, 0, s, x, ldb, L.n1, L.W, L.p, L.S, L.R);
  HIPCHK(hipGetLastError());
}

__global__ void k_extract(const double *y, int ldb, double *stM, double *stS, int n1, int W, int P, int Sw,
                          int64_t R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int lx = (int)(r % W) - P, ly = (int)((r / W) % W) - P;
  const bool inside = lx >= 0 && lx < n1 && ly >= 0 && ly < n1;
  for (int dy = -P; dy <= P; ++dy)
    for (int dx = -P; dx <= P; ++dx) {
      const int d = (dy + P) * Sw + (dx + P);
      const int nx = lx + dx, ny = ly + dy;
      double vm = 0.0, vs = 0.0;
      if (inside && nx >= 0 && nx < n1 && ny >= 0 && ny < n1) {
        const int colour = (ny % Sw) * Sw + (nx % Sw);
        vm = y[r * ldb + colour];
        vs = y[r * ldb + Sw * Sw + colour];
      }
      stM[r * Sw * Sw + d] = vm;
      stS[r * Sw * Sw + d] = vs;
    }
}

void launch_extract_stencil(const Level &L, const double *y, int ldb, double *stM, double *stS, hipStream_t s) {
  hipLaunchKernelGGL(k_extract, dim3((unsigned)((L.R + 255) / 256)), dim3(256), 0, s, y, ldb, stM, stS, L.n1, L.W,
                     L.p, L.S, L.R);
  HIPCHK(hipGetLastError());
}

// diagonals: the stencil centre of every copy, then summed over the copies of shared unknowns
// Ghost rows (outside every patch grid) get dM = 1, dS = 0: their D = sigma is positive, so the
// streaming kernels may run over ghost rows, whose vector entries stay zero.
__global__ void k_diag_centre(const double *stM, const double *stS, double *dM, double *dS, int64_t R, int c, int W,
                              int n1) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int lx = (int)(r % W) - c, ly = (int)((r / W) % W) - c;
  if (lx < 0 || lx >= n1 || ly < 0 || ly >= n1) {
    dM[r] = 1.0;
    dS[r] = 0.0;
    return;
  }
  dM[r] = stM[r * (2 * c + 1) * (2 * c + 1) + c * (2 * c + 1) + c];
  dS[r] = stS[r * (2 * c + 1) * (2 * c + 1) + c * (2 * c + 1) + c];
}
__global__ void k_diag_sum(double *dM, double *dS, const int *gp, const int *gr, int ng) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  double sm = 0, ss = 0;
  for (int k = gp[g]; k < gp[g + 1]; ++k) { sm += dM[gr[k]]; ss += dS[gr[k]]; }
  for (int k = gp[g]; k < gp[g + 1]; ++k) { dM[gr[k]] = sm; dS[gr[k]] = ss; }
}
__global__ void k_to_f32(const double *a, float *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

void launch_stencil_diag(const Level &L, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_centre, dim3((unsigned)((L.R + 255) / 256)), dim3(256), 0, s, L.stM.p, L.stS.p, L.dM.p,
                     L.dS.p, L.R, L.p, L.W, L.n1);
  if (L.ngroups > 0)
    hipLaunchKernelGGL(k_diag_sum, dim3((L.ngroups + 255) / 256), dim3(256), 0, s, L.dM.p, L.dS.p, L.grp_ptr.p,
                       L.grp_rows.p, L.ngroups);
  HIPCHK(hipGetLastError());
}

void launch_to_f32(const double *a, float *b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ white noise (Sec. 3.3)
// Pass 1, one thread per element: element mass matrix M_e = sum_q m_q phi_i phi_j, its lower
// Cholesky factor, and y_e = L_e z_e for every sample.
template <int P, int Q>
__global__ void k_noise_elements(const double *metric, const double *basis, const double *z, double *ye, int nel,
                                 int nsamp, int np) {
  constexpr int NB = P + 1, NL = NB * NB;
  const int64_t ne_tot = (int64_t)np * nel * nel;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne_tot) return;
  const int ex = (int)(e % nel), ey = (int)((e / nel) % nel);
  const double *Bx = basis + (size_t)ex * 2 * Q * NB;
  const double *By = basis + (size_t)ey * 2 * Q * NB;
  const double *mt = metric + e * Q * Q * 4;
  double A[NL][NL];
  for (int i = 0; i < NL; ++i)
    for (int j = 0; j < NL; ++j) A[i][j] = 0.0;
  for (int qy = 0; qy < Q; ++qy)
    for (int qx = 0; qx < Q; ++qx) {
      const double w = mt[(qy * Q + qx) * 4];
      double phi[NL];
      for (int b = 0; b < NB; ++b)
        for (int a = 0; a < NB; ++a) phi[b * NB + a] = By[qy * NB + b] * Bx[qx * NB + a];
      for (int i = 0; i < NL; ++i)
        for (int j = 0; j < NL; ++j) A[i][j] += w * phi[i] * phi[j];
    }
  // in-place lower Cholesky
  for (int j = 0; j < NL; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
    d = sqrt(d);
    A[j][j] = d;
    for (int i = j + 1; i < NL; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
      A[i][j] = v / d;
    }
  }
  for (int s = 0; s < nsamp; ++s) {
    const double *zs = z + ((size_t)s * ne_tot + e) * NL;
    double *ys = ye + ((size_t)s * ne_tot + e) * NL;
    for (int i = 0; i < NL; ++i) {
      double v = 0.0;
      for (int k = 0; k <= i; ++k) v += A[i][k] * zs[k];
      ys[i] = v;
    }
  }
}

// Pass 2, one thread per (coefficient row, sample): gather the element contributions of all
// elements containing the coefficient (patch-local, before the interface sum).
__global__ void k_noise_gather(const double *ye, double *bl, int nel, int n1, int W, int P, int nsamp, int64_t R,
                               int ldb, int np) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= R * nsamp) return;
  const int64_t r = id / nsamp;
  const int s = (int)(id % nsamp);
  const int lx = (int)(r % W) - P, ly = (int)((r / W) % W) - P, m = (int)(r / ((int64_t)W * W));
  if (lx < 0 || lx >= n1 || ly < 0 || ly >= n1) return;
  const int NB = P + 1, NL = NB * NB;
  const int64_t ne_tot = (int64_t)np * nel * nel;
  double v = 0.0;
  for (int b = 0; b < NB; ++b) {
    const int ey = ly - b;
    if (ey < 0 || ey >= nel) continue;
    for (int a = 0; a < NB; ++a) {
      const int ex = lx - a;
      if (ex < 0 || ex >= nel) continue;
      const int64_t e = ((int64_t)m * nel + ey) * nel + ex;
      v += ye[((size_t)s * ne_tot + e) * NL + b * NB + a];
    }
  }
  bl[r * ldb + s] = v;
}

void launch_white_noise(const Level &L, const double *z, int nsamp, double *ye, double *bl, int ldb, hipStream_t s) {
  const int64_t ne_tot = (int64_t)L.npatch * L.nel * L.nel;
  dim3 g1((unsigned)((ne_tot + 63) / 64)), b1(64);
  if (L.q != L.p + 1 && L.q != L.p + 2) fail(GF_EUNSUPPORTED, "quadrature order out of range");
  const bool q2 = L.q == L.p + 2;
  switch (L.p) {
#define GF_NE(PP)                                                                                            \
  case PP:                                                                                                   \
    if (q2)                                                                                                  \
      hipLaunchKernelGGL((k_noise_elements<PP, PP + 2>), g1, b1, 0, s, L.metric.p, L.basis.p, z, ye, L.nel, nsamp, \
                         L.npatch);                                                                          \
    else                                                                                                     \
      hipLaunchKernelGGL((k_noise_elements<PP, PP + 1>), g1, b1, 0, s, L.metric.p, L.basis.p, z, ye, L.nel, nsamp, \
                         L.npatch);                                                                          \
    break;
    GF_NE(1) GF_NE(2) GF_NE(3) GF_NE(4) GF_NE(5)
#undef GF_NE
    default: fail(GF_EUNSUPPORTED, "degree out of range");
  }
  HIPCHK(hipGetLastError());
  const int64_t tot = L.R * nsamp;
  hipLaunchKernelGGL(k_noise_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ye, bl, L.nel, L.n1, L.W,
                     L.p, nsamp, L.R, ldb, L.npatch);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ coarse Cholesky
// One thread per node: A = sigma M0 + S0 (dense, global numbering of the coarsest level),
// lower Cholesky factor in place.  info = 0 on success, k+1 if pivot k is not positive.
__global__ void k_coarse_factor(const double *M0, const double *S0, int n, const double *sig, int nnode, double *Lf,
                                int *info) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnode) return;
  double *A = Lf + (size_t)k * n * n;
  const double sg = sig[k];
  for (int i = 0; i < n * n; ++i) A[i] = sg * M0[i] + S0[i];
  int bad = 0;
  for (int j = 0; j < n && !bad; ++j) {
    double d = A[j * n + j];
    for (int t = 0; t < j; ++t) d -= A[j * n + t] * A[j * n + t];
    if (!(d > 0.0)) { bad = j + 1; break; }
    d = sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int t = 0; t < j; ++t) v -= A[i * n + t] * A[j * n + t];
      A[i * n + j] = v / d;
    }
    for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;  // clear the upper triangle
  }
  info[k] = bad;
}

void launch_coarse_factor(const double *M0, const double *S0, int N0, const double *sig, int nnode, double *Lf,
                          int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_factor, dim3((nnode + 63) / 64), dim3(64), 0, s, M0, S0, N0, sig, nnode, Lf, info);
  HIPCHK(hipGetLastError());
}

// A^-1 = L^-T L^-1 from the Cholesky factor, one block per node, thread j builds column j:
// forward substitution L y = e_j, then back substitution L^T x = y, both in place in the column.
__global__ void k_coarse_inverse(const double *Lf, int n, int nnode, double *Ainv) {
  const int k = blockIdx.x;
  if (k >= nnode) return;
  const double *L = Lf + (size_t)k * n * n;
  double *X = Ainv + (size_t)k * n * n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int t = j; t < i; ++t) s -= L[(size_t)i * n + t] * X[(size_t)t * n + j];
      X[(size_t)i * n + j] = (i < j) ? 0.0 : s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = X[(size_t)i * n + j];
      for (int t = i + 1; t < n; ++t) s -= L[(size_t)t * n + i] * X[(size_t)t * n + j];
      X[(size_t)i * n + j] = s / L[(size_t)i * n + i];
    }
  }
}

void launch_coarse_inverse(const double *Lf, int N0, int nnode, double *Ainv, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_inverse, dim3(nnode), dim3(std::min(1024, (N0 + 63) / 64 * 64)), 0, s, Lf, N0, nnode,
                     Ainv);
  HIPCHK(hipGetLastError());
}

}  // namespace gf
