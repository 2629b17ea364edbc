// Point evaluation of spline fields, its transpose, and the per-sample accumulation of the
// kappa-gradient terms.
//
// A field of S^0_{j,p} restricted to patch m is the tensor spline sum c[m,iy,ix] b_ix(s) b_iy(t)
// (Sec. 2.3, Sec. 3.1); its value at the surface point F_m(s,t) is that sum, so evaluation at a set of
// points is a sparse matrix Phi with (p+1)^2 entries per point.  The basis values come from the
// triangular Cox-de Boor scheme on the open dyadic knot vector (p+1-fold end knots, interior knots
// i 2^-j), evaluated on the device for every point.
#include "gf_internal.h"
#include "k_solve.h"

namespace gf {

// knot i of the open uniform knot vector with nel elements and degree p
__device__ __forceinline__ double knot_at(int i, int p, int nel) {
  const int k = min(max(i - p, 0), nel);
  return (double)k / (double)nel;
}

// The p+1 B-splines of degree p that are nonzero on the element containing u (the last element
// for u = 1): values into N[0..p] for the functions e..e+p; returns e.
template <int MAXP>
__device__ int span_basis(double u, int p, int nel, double *N) {
  int e = (int)floor(u * nel);
  e = min(max(e, 0), nel - 1);
  const int span = e + p;  // knot interval [knot(span), knot(span + 1))
  double left[MAXP + 1], right[MAXP + 1];
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = u - knot_at(span + 1 - j, p, nel);
    right[j] = knot_at(span + j, p, nel) - u;
    double carry = 0.0;
    for (int r = 0; r < j; ++r) {
      const double den = right[r + 1] + left[j - r];
      const double t = den != 0.0 ? N[r] / den : 0.0;
      N[r] = carry + right[r + 1] * t;
      carry = left[j - r] * t;
    }
    N[j] = carry;
  }
  return e;
}

struct EvalGeom {
  int p, nel, W, N, npts, nvec;
};

// vals[v][i] = sum over the (p+1)^2 basis functions of point i of B(s_i, t_i) u[v][gid]
__global__ __launch_bounds__(256) void k_eval(EvalGeom g, const int *__restrict__ patch, const double *__restrict__ st,
                                              const int *__restrict__ row_gid, const double *__restrict__ u,
                                              double *__restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.npts) return;
  double bs[6], bt[6];
  const int ex = span_basis<5>(st[2 * i], g.p, g.nel, bs);
  const int ey = span_basis<5>(st[2 * i + 1], g.p, g.nel, bt);
  const int64_t base = (int64_t)patch[i] * g.W * g.W;
  int gid[36];
  for (int a = 0; a <= g.p; ++a)
    for (int b = 0; b <= g.p; ++b)
      gid[a * (g.p + 1) + b] = row_gid[base + (int64_t)(ey + a + g.p) * g.W + (ex + b + g.p)];
  for (int v = 0; v < g.nvec; ++v) {
    const double *uv = u + (int64_t)v * g.N;
    double acc = 0.0;
    for (int a = 0; a <= g.p; ++a) {
      double ra = 0.0;
      for (int b = 0; b <= g.p; ++b) ra += bs[b] * uv[gid[a * (g.p + 1) + b]];
      acc += bt[a] * ra;
    }
    vals[(int64_t)v * g.npts + i] = acc;
  }
}

// The transpose Phi^T r without atomics, in two passes.  Pass 1: the (p+1)^2 basis products of every
// point, w[i][a (p+1) + b] = B_a(t_i) B_b(s_i).  Pass 2: one thread per (global coefficient, vector)
// sums w r over the entries the host listed for that coefficient, in ascending point order: the
// result does not depend on the scheduling and is the same bit for bit on every run.
__global__ __launch_bounds__(256) void k_eval_weights(EvalGeom g, const double *__restrict__ st, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.npts) return;
  double bs[6], bt[6];
  span_basis<5>(st[2 * i], g.p, g.nel, bs);
  span_basis<5>(st[2 * i + 1], g.p, g.nel, bt);
  const int nb = g.p + 1;
  for (int a = 0; a <= g.p; ++a)
    for (int b = 0; b <= g.p; ++b) w[(int64_t)i * nb * nb + a * nb + b] = bt[a] * bs[b];
}

// out[v][gid] = sum over the entries e of gid (ptr[gid] .. ptr[gid+1], ascending point order) of
// w[ent[e]] r[v][ent[e] / (p+1)^2]; coefficients no point touches get 0
__global__ __launch_bounds__(256) void k_eval_gather(EvalGeom g, const int *__restrict__ ptr, const int *__restrict__ ent,
                                                     const double *__restrict__ w, const double *__restrict__ r,
                                                     double *__restrict__ out) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)g.N * g.nvec) return;
  const int gid = (int)(id % g.N), v = (int)(id / g.N);
  const int nb2 = (g.p + 1) * (g.p + 1);
  double acc = 0.0;
  for (int e = ptr[gid]; e < ptr[gid + 1]; ++e) {
    const int k = ent[e];
    acc += w[k] * r[(int64_t)v * g.npts + k / nb2];
  }
  out[(int64_t)v * g.N + gid] = acc;
}

void launch_eval(const Level &L, int npts, const int *patch, const double *st, int nvec, const double *u,
                 double *vals, hipStream_t s) {
  if (npts == 0 || nvec == 0) return;
  EvalGeom g{L.p, L.nel, L.W, L.N, npts, nvec};
  hipLaunchKernelGGL(k_eval, dim3((npts + 255) / 256), dim3(256), 0, s, g, patch, st, L.row_gid.p, u, vals);
  HIPCHK(hipGetLastError());
}

void launch_eval_adjoint(const Level &L, int npts, const double *st, const int *ptr, const int *ent, double *w,
                         int nvec, const double *r, double *out, hipStream_t s) {
  if (nvec == 0) return;
  EvalGeom g{L.p, L.nel, L.W, L.N, npts, nvec};
  if (npts > 0) hipLaunchKernelGGL(k_eval_weights, dim3((npts + 255) / 256), dim3(256), 0, s, g, st, w);
  const int64_t tot = (int64_t)L.N * nvec;
  hipLaunchKernelGGL(k_eval_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g, ptr, ent, w, r, out);
  HIPCHK(hipGetLastError());
}

// acc[s] += sum_k w[k] dots[k * nsamp + s], k ascending (one thread per sample)
__global__ void k_grad_accum(const double *__restrict__ dots, const double *__restrict__ w, int K, int nsamp,
                             double *acc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsamp) return;
  double t = 0.0;
  for (int k = 0; k < K; ++k) t += w[k] * dots[(int64_t)k * nsamp + s];
  acc[s] += t;
}

// out[s] = c * acc[s]
__global__ void k_grad_scale(const double *__restrict__ acc, int nsamp, double c, double *out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsamp) out[s] = c * acc[s];
}

void grad_accum(const double *dots, const double *w, int K, int nsamp, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_accum, dim3((nsamp + 255) / 256), dim3(256), 0, s, dots, w, K, nsamp, acc);
  HIPCHK(hipGetLastError());
}

void grad_scale(const double *acc, int nsamp, double c, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_scale, dim3((nsamp + 255) / 256), dim3(256), 0, s, acc, nsamp, c, out);
  HIPCHK(hipGetLastError());
}

}  // namespace gf
