// Solver kernels: stencil operator application, interface sums, wavefront-reduction
// inner products with per-system CG scalar updates, CG vector updates, Chebyshev-Jacobi
// smoothing, knot-insertion transfers, the coarsest-level Cholesky solve, and the
// conversions between the caller's global numbering and the patch-local batch layout.
//
// Batch layout (all kernels): rows of the padded patch-local grid, 64-column tiles of
// systems; one wavefront covers one row of one tile, lane = system, so per-row data
// (stencils, diagonals, masks) is uniform over the wavefront and every vector access is
// a contiguous 256 B (FP32) or 512 B (FP64) transaction.
#include "gf_internal.h"
#include "k_solve.h"

namespace gf {

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ bool row_interior(int64_t r, int W, int P, int n1) {
  const int lx = (int)(r % W) - P, ly = (int)((r / W) % W) - P;
  return lx >= 0 && lx < n1 && ly >= 0 && ly < n1;
}

// ------------------------------------------------------------------ interface sum
// Copies of one unknown on neighbouring patches (2 on edges, 3 at cube corners) receive the
// sum of their patch contributions: this turns patch-local results into the assembled
// global operator (Sec. 2.3, continuity across interfaces).
template <typename T>
__global__ __launch_bounds__(256) void k_iface(T *y, int ldb, const int *__restrict__ gp, const int *__restrict__ gr,
                                               int ng, const int *__restrict__ active) {
  const int ntiles = ldb / CT;
  const int ct = blockIdx.x % ntiles;
  if (active && !active[ct]) return;
  const int g = wave_uniform((int)(blockIdx.x / ntiles) * 4 + threadIdx.y);
  if (g >= ng) return;
  const int col = ct * CT + threadIdx.x;
  const int k0 = gp[g], k1 = gp[g + 1];
  T s = 0;
  for (int k = k0; k < k1; ++k) s += y[(int64_t)gr[k] * ldb + col];
  for (int k = k0; k < k1; ++k) y[(int64_t)gr[k] * ldb + col] = s;
}

template <typename T>
void launch_interface_sum(const Level &L, T *y, int ldb, int ntiles, const int *active, hipStream_t s) {
  if (L.ngroups == 0) return;
  hipLaunchKernelGGL(k_iface<T>, dim3(ntiles * ((L.ngroups + 3) / 4)), dim3(CT, 4), 0, s, y, ldb, L.grp_ptr.p,
                     L.grp_rows.p, L.ngroups, active);
  HIPCHK(hipGetLastError());
}
template void launch_interface_sum<double>(const Level &, double *, int, int, const int *, hipStream_t);
template void launch_interface_sum<float>(const Level &, float *, int, int, const int *, hipStream_t);

// ------------------------------------------------------------------ reductions
// Row-loop kernels with an inner-product epilogue.  Each block reduces its rows for the 64
// columns of its tile through LDS, writes one partial per column, and the last block of the
// tile to finish (device-scope counter) sums the partials in block order -- a fixed order,
// so results are bitwise reproducible -- and applies the per-system scalar step `op`.
struct RowCtx {
  int64_t R;
  int W, P, n1, ldb;
  const uint8_t *owner;
};

template <class F, int ND>
__global__ __launch_bounds__(256) void k_rowreduce(F f, RowCtx rc, double *partial, const int *active) {
  const int ct = blockIdx.x;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x;
  const int col = ct * CT + lane;
  const int wave = wave_uniform(threadIdx.y);
  double acc[ND];
#pragma unroll
  for (int k = 0; k < ND; ++k) acc[k] = 0.0;
  for (int64_t r = (int64_t)blockIdx.y * 4 + wave; r < rc.R; r += (int64_t)gridDim.y * 4) f(r, col, rc.owner[r] != 0, acc);
  __shared__ double red[4][ND][CT];
#pragma unroll
  for (int k = 0; k < ND; ++k) red[threadIdx.y][k][lane] = acc[k];
  __syncthreads();
  if (threadIdx.y != 0) return;
  const int nrb = gridDim.y;
#pragma unroll
  for (int k = 0; k < ND; ++k)
    partial[((int64_t)k * nrb + blockIdx.y) * rc.ldb + col] =
        red[0][k][lane] + red[1][k][lane] + red[2][k][lane] + red[3][k][lane];
}

// row functors ------------------------------------------------------
template <typename TA, typename TB>
struct FDot {
  const TA *a;
  const TB *b;
  int ldb;
  __device__ void operator()(int64_t r, int col, bool own, double *acc) const {
    if (own) acc[0] += (double)a[r * ldb + col] * (double)b[r * ldb + col];
  }
};
template <typename TA, typename TB, typename TC>
struct FDot2 {  // acc0 = a.b, acc1 = b.c
  const TA *a;
  const TB *b;
  const TC *c;
  int ldb;
  __device__ void operator()(int64_t r, int col, bool own, double *acc) const {
    if (own) {
      const double bv = (double)b[r * ldb + col];
      acc[0] += (double)a[r * ldb + col] * bv;
      acc[1] += bv * (double)c[r * ldb + col];
    }
  }
};

static RowCtx rowctx(const Level &L, int ldb) { return RowCtx{L.R, L.W, L.p, L.n1, ldb, L.owner.p}; }

static int row_blocks(const Level &L, int ntiles) {
  const int64_t waves_rows = (L.R + 3) / 4;
  int nrb = (int)std::min<int64_t>(waves_rows, std::max<int64_t>(1, 4096 / std::max(1, ntiles)));
  return std::max(1, std::min(nrb, kMaxRowBlocks));
}

template <class F, int ND>
static void run_reduce(const Level &L, F f, Scratch &sc, int ldb, int ntiles, ColState *cs, int *active, int op,
                       double tol2, int maxit, double *out, hipStream_t s) {
  const int nrb = row_blocks(L, ntiles);
  hipLaunchKernelGGL((k_rowreduce<F, ND>), dim3(ntiles, nrb), dim3(CT, 4), 0, s, f, rowctx(L, ldb), sc.partial,
                     active);
  HIPCHK(hipGetLastError());
  finalize(nrb, ND, op, sc, cs, active, ldb, ntiles, tol2, maxit, out, s);
}

template <typename TA, typename TB>
void reduce_dot(const Level &L, const TA *a, const TB *b, Scratch &sc, int ldb, int ntiles, ColState *cs,
                int *active, int op, double tol2, int maxit, double *out, hipStream_t s) {
  run_reduce<FDot<TA, TB>, 1>(L, FDot<TA, TB>{a, b, ldb}, sc, ldb, ntiles, cs, active, op, tol2, maxit, out, s);
}
template void reduce_dot<double, double>(const Level &, const double *, const double *, Scratch &, int, int,
                                         ColState *, int *, int, double, int, double *, hipStream_t);
template void reduce_dot<double, float>(const Level &, const double *, const float *, Scratch &, int, int,
                                        ColState *, int *, int, double, int, double *, hipStream_t);

template <typename TA, typename TB, typename TC>
void reduce_dot2(const Level &L, const TA *a, const TB *b, const TC *c, Scratch &sc, int ldb, int ntiles,
                 ColState *cs, int *active, int op, double tol2, int maxit, double *out, hipStream_t s) {
  run_reduce<FDot2<TA, TB, TC>, 2>(L, FDot2<TA, TB, TC>{a, b, c, ldb}, sc, ldb, ntiles, cs, active, op, tol2, maxit,
                                   out, s);
}
template void reduce_dot2<double, double, double>(const Level &, const double *, const double *, const double *,
                                                  Scratch &, int, int, ColState *, int *, int, double, int, double *,
                                                  hipStream_t);
template void reduce_dot2<double, float, double>(const Level &, const double *, const float *, const double *,
                                                 Scratch &, int, int, ColState *, int *, int, double, int, double *,
                                                 hipStream_t);


// ------------------------------------------------------------------ elementwise row kernels
template <class F>
__global__ __launch_bounds__(256) void k_rows(F f, RowCtx rc, const int *__restrict__ active) {
  const int ct = blockIdx.x;
  if (active && !active[ct]) return;
  const int col = ct * CT + threadIdx.x;
  const int wave = wave_uniform(threadIdx.y);
  for (int64_t r = (int64_t)blockIdx.y * 4 + wave; r < rc.R; r += (int64_t)gridDim.y * 4) {
    if (!row_interior(r, rc.W, rc.P, rc.n1)) continue;
    f(r, col);
  }
}

template <class F>
static void run_rows(const Level &L, F f, int ldb, int ntiles, const int *active, hipStream_t s) {
  const int nrb = row_blocks(L, ntiles);
  hipLaunchKernelGGL(k_rows<F>, dim3(ntiles, nrb), dim3(CT, 4), 0, s, f, rowctx(L, ldb), active);
  HIPCHK(hipGetLastError());
}


template <typename TS, typename TD>
struct FConvert {
  const TS *a;
  TD *b;
  int ldb;
  __device__ void operator()(int64_t r, int col) const { b[r * ldb + col] = (TD)a[r * ldb + col]; }
};
template <typename TS, typename TD>
void convert_rows(const Level &L, const TS *a, TD *b, int ldb, int ntiles, const int *active, hipStream_t s) {
  run_rows(L, FConvert<TS, TD>{a, b, ldb}, ldb, ntiles, active, s);
}
template void convert_rows<double, float>(const Level &, const double *, float *, int, int, const int *,
                                          hipStream_t);
template void convert_rows<float, double>(const Level &, const float *, double *, int, int, const int *,
                                          hipStream_t);
template void convert_rows<double, double>(const Level &, const double *, double *, int, int, const int *,
                                           hipStream_t);
template void convert_rows<float, float>(const Level &, const float *, float *, int, int, const int *, hipStream_t);

// power-iteration step for the spectral bound of D^-1 A: v = w / D
struct FDivDiag {
  double *v;
  const double *w, *dM, *dS, *sig;
  int ldb;
  __device__ void operator()(int64_t row, int col) const {
    const int64_t i = row * ldb + col;
    v[i] = w[i] / (sig[col] * dM[row] + dS[row]);
  }
};
void div_diag(const Level &L, double *v, const double *w, const double *sig, int ldb, int ntiles, hipStream_t s) {
  run_rows(L, FDivDiag{v, w, L.dM.p, L.dS.p, sig, ldb}, ldb, ntiles, nullptr, s);
}

// v = w / (ca dA + cb dB) with per-column ca, cb and per-row diagonals dA, dB
struct FDivDiag2 {
  double *v;
  const double *w, *ca, *dA, *cb, *dB;
  int ldb;
  __device__ void operator()(int64_t row, int col) const {
    const int64_t i = row * ldb + col;
    v[i] = w[i] / (ca[col] * dA[row] + cb[col] * dB[row]);
  }
};
void div_diag2(const Level &L, double *v, const double *w, const double *ca, const double *dA, const double *cb,
               const double *dB, int ldb, int ntiles, const int *active, hipStream_t s) {
  run_rows(L, FDivDiag2{v, w, ca, dA, cb, dB, ldb}, ldb, ntiles, active, s);
}

// z = r / (sig dM + dS): the diagonal scaling of one level of the additive multilevel preconditioner
template <typename T>
struct FDiagScale {
  T *z;
  const T *r, *sig, *dM, *dS;
  int ldb;
  __device__ void operator()(int64_t row, int col) const {
    const int64_t i = row * ldb + col;
    z[i] = r[i] / (sig[col] * dM[row] + dS[row]);
  }
};
template <typename T>
void diag_scale(const Level &L, T *z, const T *r, const T *sig, const T *dM, const T *dS, int ldb, int ntiles,
                const int *active, hipStream_t s) {
  run_rows(L, FDiagScale<T>{z, r, sig, dM, dS, ldb}, ldb, ntiles, active, s);
}
template void diag_scale<double>(const Level &, double *, const double *, const double *, const double *,
                                 const double *, int, int, const int *, hipStream_t);
template void diag_scale<float>(const Level &, float *, const float *, const float *, const float *, const float *,
                                int, int, const int *, hipStream_t);

// deterministic start vector in [0.5, 1.5) from a hash of (row, column)
struct FHashFill {
  double *v;
  int ldb;
  __device__ void operator()(int64_t row, int col) const {
    uint64_t h = (uint64_t)row * 0x9E3779B97F4A7C15ull ^ ((uint64_t)col + 0x632BE59BD9B4E019ull);
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 27;
    h *= 0x94D049BB133111EBull;
    h ^= h >> 31;
    v[row * ldb + col] = 0.5 + (double)(h >> 11) * (1.0 / 9007199254740992.0);
  }
};
void hash_fill(const Level &L, double *v, int ldb, int ntiles, hipStream_t s) {
  run_rows(L, FHashFill{v, ldb}, ldb, ntiles, nullptr, s);
}

// ------------------------------------------------------------------ transfers
// Restriction of a residual: rc = P^T (owner mask (r - Az)) per patch, 1D knot-insertion
// matrices in both directions (tensor product).  The owner mask turns the assembled fine
// residual into one contribution per unknown; the coarse interface sum follows.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(T *rc, const T *r, const T *Az, const uint8_t *__restrict__ ownf,
                                                  int Wf, int Wc, int n1c, int P, int ldb,
                                                  const int *__restrict__ rs, const T *__restrict__ rcoef, int rw,
                                                  const int *__restrict__ active, int ntiles, int np) {
  const int ct = blockIdx.x % ntiles;
  if (active && !active[ct]) return;
  const int col = ct * CT + threadIdx.x;
  const int id = wave_uniform((int)(blockIdx.x / ntiles) * 4 + threadIdx.y);
  if (id >= np * n1c * n1c) return;
  const int ixc = id % n1c, iyc = (id / n1c) % n1c, m = id / (n1c * n1c);
  const int64_t fbase = (int64_t)m * Wf * Wf;
  const int fy0 = rs[iyc], fx0 = rs[ixc];
  T acc = 0;
  for (int k = 0; k < rw; ++k) {
    const T wy = rcoef[iyc * rw + k];
    if (wy == T(0)) continue;
    for (int l = 0; l < rw; ++l) {
      const T wx = rcoef[ixc * rw + l];
      if (wx == T(0)) continue;
      const int64_t rf = fbase + (int64_t)(fy0 + k + P) * Wf + (fx0 + l + P);
      if (!ownf[rf]) continue;
      const int64_t i = rf * ldb + col;
      acc += wy * wx * (Az ? r[i] - Az[i] : r[i]);
    }
  }
  rc[((int64_t)m * Wc * Wc + (int64_t)(iyc + P) * Wc + (ixc + P)) * ldb + col] = acc;
}

// Prolongation: zf += P zc (knot insertion, tensor product per patch).
template <typename T>
__global__ __launch_bounds__(256) void k_prolong(T *zf, const T *zc, int Wf, int Wc, int n1f, int P, int ldb,
                                                 const int *__restrict__ ps, const T *__restrict__ pcoef, int pw,
                                                 const int *__restrict__ active, int ntiles, int np) {
  const int ct = blockIdx.x % ntiles;
  if (active && !active[ct]) return;
  const int col = ct * CT + threadIdx.x;
  const int id = wave_uniform((int)(blockIdx.x / ntiles) * 4 + threadIdx.y);
  if (id >= np * n1f * n1f) return;
  const int ixf = id % n1f, iyf = (id / n1f) % n1f, m = id / (n1f * n1f);
  const int64_t cbase = (int64_t)m * Wc * Wc;
  const int cy0 = ps[iyf], cx0 = ps[ixf];
  T acc = 0;
  for (int k = 0; k < pw; ++k) {
    const T wy = pcoef[iyf * pw + k];
    if (wy == T(0)) continue;
    for (int l = 0; l < pw; ++l) {
      const T wx = pcoef[ixf * pw + l];
      if (wx == T(0)) continue;
      acc += wy * wx * zc[(cbase + (int64_t)(cy0 + k + P) * Wc + (cx0 + l + P)) * ldb + col];
    }
  }
  const int64_t i = ((int64_t)m * Wf * Wf + (int64_t)(iyf + P) * Wf + (ixf + P)) * ldb + col;
  zf[i] += acc;
}

// Line-marching forms of the two transfers.  One wavefront per (patch, output row, segment of the
// row's outputs, column tile) walks the input columns of its band of input rows in order: the
// contraction across rows is done once per input column and pushed into a register window, and every
// output whose band ends at that column is formed from the window.  Each input value is thus loaded
// once per output row that needs it (instead of once per output value; a segment boundary repeats
// the few input columns of one band) and the loop body has no data-dependent branches.  The
// knot-insertion bands have fixed widths rw <= p+2 (restriction) and pw <= (p+3)/2 (prolongation)
// and start at non-decreasing input indices (rs, ps).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_restrict_rows(T *rc, const T *__restrict__ r, const uint8_t *__restrict__ ownf,
                                                       int Wf, int Wc, int n1f, int n1c, int ldb,
                                                       const int *__restrict__ rs, const T *__restrict__ rcoef, int rw,
                                                       const int *__restrict__ active, int ntiles, int np, int nseg) {
  constexpr int RW = P + 2;
  const int ct = blockIdx.x % ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x;
  const int wid = wave_uniform((int)(blockIdx.x / ntiles) * 4 + threadIdx.y);
  if (wid >= np * n1c * nseg) return;
  // segment sg of the row: outputs [c0, c1); the march starts at the first input of c0's band (the
  // register window holds only columns of the bands it forms)
  const int id = wid / nseg, sg = wid - id * nseg;
  const int seglen = (n1c + nseg - 1) / nseg;
  const int c0 = sg * seglen, c1 = min(c0 + seglen, n1c);
  if (c0 >= c1) return;
  const int iyc = id % n1c, m = id / n1c;
  const int64_t ct0 = (int64_t)ct * CT;
  const int64_t fbase = (int64_t)m * Wf * Wf;
  const int fy0 = rs[iyc];
  T wy[RW];
  int64_t frow[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    wy[k] = k < rw ? rcoef[iyc * rw + k] : T(0);
    // rows past the band carry weight 0; clamped so that their loads stay inside the patch
    frow[k] = fbase + (int64_t)(min(fy0 + k, n1f - 1) + P) * Wf + P;
  }
  const int64_t cbase = (int64_t)m * Wc * Wc + (int64_t)(iyc + P) * Wc + P;
  // one contribution per unknown: only owner copies count.  Every unknown off the patch boundary is
  // its own owner, so the owner flags are read only on boundary rows and columns.
  bool brow = false;
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    const int fy = min(fy0 + k, n1f - 1);
    brow = brow || (k < rw && (fy == 0 || fy == n1f - 1));
  }
  T tw[RW];
#pragma unroll
  for (int l = 0; l < RW; ++l) tw[l] = 0;
  int ixc = c0;
  int last = rs[c0] + rw - 1;  // last fine column of output ixc's band
  // the input column's values, loaded one column ahead of their use
  T cv[RW];
  const int fxs = rs[c0];
#pragma unroll
  for (int k = 0; k < RW; ++k) cv[k] = (r + (frow[k] + fxs) * ldb + ct0)[lane];
  for (int fx = fxs; fx < n1f && ixc < c1; ++fx) {
    const int fxn = min(fx + 1, n1f - 1);
    T nv[RW];
#pragma unroll
    for (int k = 0; k < RW; ++k) nv[k] = (r + (frow[k] + fxn) * ldb + ct0)[lane];
    T t = 0;
    if (brow || fx == 0 || fx == n1f - 1) {
#pragma unroll
      for (int k = 0; k < RW; ++k) t += (ownf[frow[k] + fx] ? wy[k] : T(0)) * cv[k];
    } else {
#pragma unroll
      for (int k = 0; k < RW; ++k) t += wy[k] * cv[k];
    }
#pragma unroll
    for (int l = 0; l < RW - 1; ++l) tw[l] = tw[l + 1];
    tw[RW - 1] = t;  // the window now holds fine columns fx-RW+1 .. fx
    while (ixc < c1 && last == fx) {
      T acc = 0;
#pragma unroll
      for (int l = 0; l < RW; ++l) {
        const int j = l - (RW - rw);
        if (j >= 0) acc += rcoef[ixc * rw + j] * tw[l];
      }
      (rc + (cbase + ixc) * ldb + ct0)[lane] = acc;
      ++ixc;
      if (ixc < c1) last = rs[ixc] + rw - 1;
    }
#pragma unroll
    for (int k = 0; k < RW; ++k) cv[k] = nv[k];
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_prolong_rows(T *zf, const T *__restrict__ zc, int Wf, int Wc, int n1f, int n1c,
                                                      int ldb, const int *__restrict__ ps,
                                                      const T *__restrict__ pcoef, int pw,
                                                      const int *__restrict__ active, int ntiles, int np, int nseg) {
  constexpr int PW = (P + 3) / 2;
  const int ct = blockIdx.x % ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x;
  const int wid = wave_uniform((int)(blockIdx.x / ntiles) * 4 + threadIdx.y);
  if (wid >= np * n1f * nseg) return;
  // segment sg of the row: outputs [f0, f1), the march starting at the first input of f0's band
  const int id = wid / nseg, sg = wid - id * nseg;
  const int seglen = (n1f + nseg - 1) / nseg;
  const int f0 = sg * seglen, f1 = min(f0 + seglen, n1f);
  if (f0 >= f1) return;
  const int iyf = id % n1f, m = id / n1f;
  const int64_t ct0 = (int64_t)ct * CT;
  const int64_t cbase = (int64_t)m * Wc * Wc;
  const int cy0 = ps[iyf];
  T wy[PW];
  int64_t crow[PW];
#pragma unroll
  for (int k = 0; k < PW; ++k) {
    wy[k] = k < pw ? pcoef[iyf * pw + k] : T(0);
    crow[k] = cbase + (int64_t)(min(cy0 + k, n1c - 1) + P) * Wc + P;
  }
  const int64_t fbase = (int64_t)m * Wf * Wf + (int64_t)(iyf + P) * Wf + P;
  T sw[PW];
#pragma unroll
  for (int l = 0; l < PW; ++l) sw[l] = 0;
  int ixf = f0;
  int last = ps[f0] + pw - 1;  // last coarse column of fine output ixf's band
  // loaded ahead of their use: the coarse values of the next input column, and the fine values of the
  // next two outputs (each is read before an earlier output is stored; they are different entries)
  const int cxs = ps[f0];
  T cv[PW];
#pragma unroll
  for (int k = 0; k < PW; ++k) cv[k] = (zc + (crow[k] + cxs) * ldb + ct0)[lane];
  T z0 = (zf + (fbase + ixf) * ldb + ct0)[lane];
  T z1 = (zf + (fbase + min(ixf + 1, f1 - 1)) * ldb + ct0)[lane];
  for (int cx = cxs; cx < n1c && ixf < f1; ++cx) {
    const int cxn = min(cx + 1, n1c - 1);
    T nv[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) nv[k] = (zc + (crow[k] + cxn) * ldb + ct0)[lane];
    T t = 0;
#pragma unroll
    for (int k = 0; k < PW; ++k) t += wy[k] * cv[k];
#pragma unroll
    for (int l = 0; l < PW - 1; ++l) sw[l] = sw[l + 1];
    sw[PW - 1] = t;
    while (ixf < f1 && last == cx) {
      T acc = 0;
#pragma unroll
      for (int l = 0; l < PW; ++l) {
        const int j = l - (PW - pw);
        if (j >= 0) acc += pcoef[ixf * pw + j] * sw[l];
      }
      const T z2 = (zf + (fbase + min(ixf + 2, f1 - 1)) * ldb + ct0)[lane];
      (zf + (fbase + ixf) * ldb + ct0)[lane] = z0 + acc;
      z0 = z1;
      z1 = z2;
      ++ixf;
      if (ixf < f1) last = ps[ixf] + pw - 1;
    }
#pragma unroll
    for (int k = 0; k < PW; ++k) cv[k] = nv[k];
  }
}

// Segments per output row of the line-marching transfers: enough wavefronts (4096) for the chip when
// the batch has few column tiles, at most eight (each segment re-marches the band of its first output)
static int transfer_segments(int rows, int ntiles) {
  const int64_t waves = (int64_t)rows * ntiles;
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, (4096 + waves - 1) / std::max<int64_t>(1, waves)));
}

template <typename T>
static const T *res_coef(const Level &F);
template <>
const double *res_coef<double>(const Level &F) { return F.res_c.p; }
template <>
const float *res_coef<float>(const Level &F) { return F.res_c32.p; }
template <typename T>
static const T *pro_coef(const Level &F);
template <>
const double *pro_coef<double>(const Level &F) { return F.pro_c.p; }
template <>
const float *pro_coef<float>(const Level &F) { return F.pro_c32.p; }

template <typename T, int P>
static void launch_restrict_rows(const Level &F, const Level &C, T *rc, const T *r, int ldb, int ntiles,
                                 const int *active, hipStream_t s) {
  const int nseg = transfer_segments(F.npatch * C.n1, ntiles);
  const int n = F.npatch * C.n1 * nseg;
  hipLaunchKernelGGL((k_restrict_rows<T, P>), dim3(ntiles * ((n + 3) / 4)), dim3(CT, 4), 0, s, rc, r, F.owner.p, F.W,
                     C.W, F.n1, C.n1, ldb, F.res_start.p, res_coef<T>(F), F.rw, active, ntiles, F.npatch, nseg);
}

template <typename T>
void restrict_residual(const Level &F, const Level &C, T *rc, const T *r, const T *Az, int ldb, int ntiles,
                       const int *active, hipStream_t s) {
  if (Az == nullptr && F.rw <= F.p + 2) {
    switch (F.p) {
      case 1: launch_restrict_rows<T, 1>(F, C, rc, r, ldb, ntiles, active, s); break;
      case 2: launch_restrict_rows<T, 2>(F, C, rc, r, ldb, ntiles, active, s); break;
      case 3: launch_restrict_rows<T, 3>(F, C, rc, r, ldb, ntiles, active, s); break;
      case 4: launch_restrict_rows<T, 4>(F, C, rc, r, ldb, ntiles, active, s); break;
      default: launch_restrict_rows<T, 5>(F, C, rc, r, ldb, ntiles, active, s); break;
    }
  } else {
    const int n = F.npatch * C.n1 * C.n1;
    hipLaunchKernelGGL(k_restrict<T>, dim3(ntiles * ((n + 3) / 4)), dim3(CT, 4), 0, s, rc, r, Az, F.owner.p, F.W,
                       C.W, C.n1, F.p, ldb, F.res_start.p, res_coef<T>(F), F.rw, active, ntiles, F.npatch);
  }
  HIPCHK(hipGetLastError());
}
template void restrict_residual<double>(const Level &, const Level &, double *, const double *, const double *, int,
                                        int, const int *, hipStream_t);
template void restrict_residual<float>(const Level &, const Level &, float *, const float *, const float *, int, int,
                                       const int *, hipStream_t);

template <typename T, int P>
static void launch_prolong_rows(const Level &F, const Level &C, T *zf, const T *zc, int ldb, int ntiles,
                                const int *active, hipStream_t s) {
  const int nseg = transfer_segments(F.npatch * F.n1, ntiles);
  const int n = F.npatch * F.n1 * nseg;
  hipLaunchKernelGGL((k_prolong_rows<T, P>), dim3(ntiles * ((n + 3) / 4)), dim3(CT, 4), 0, s, zf, zc, F.W, C.W, F.n1,
                     C.n1, ldb, F.pro_start.p, pro_coef<T>(F), F.pw, active, ntiles, F.npatch, nseg);
}

template <typename T>
void prolong_add(const Level &F, const Level &C, T *zf, const T *zc, int ldb, int ntiles, const int *active,
                 hipStream_t s) {
  if (F.pw <= (F.p + 3) / 2) {
    switch (F.p) {
      case 1: launch_prolong_rows<T, 1>(F, C, zf, zc, ldb, ntiles, active, s); break;
      case 2: launch_prolong_rows<T, 2>(F, C, zf, zc, ldb, ntiles, active, s); break;
      case 3: launch_prolong_rows<T, 3>(F, C, zf, zc, ldb, ntiles, active, s); break;
      case 4: launch_prolong_rows<T, 4>(F, C, zf, zc, ldb, ntiles, active, s); break;
      default: launch_prolong_rows<T, 5>(F, C, zf, zc, ldb, ntiles, active, s); break;
    }
  } else {
    const int n = F.npatch * F.n1 * F.n1;
    hipLaunchKernelGGL(k_prolong<T>, dim3(ntiles * ((n + 3) / 4)), dim3(CT, 4), 0, s, zf, zc, F.W, C.W, F.n1, F.p,
                       ldb, F.pro_start.p, pro_coef<T>(F), F.pw, active, ntiles, F.npatch);
  }
  HIPCHK(hipGetLastError());
}
template void prolong_add<double>(const Level &, const Level &, double *, const double *, int, int, const int *,
                                  hipStream_t);
template void prolong_add<float>(const Level &, const Level &, float *, const float *, int, int, const int *,
                                 hipStream_t);

// ------------------------------------------------------------------ coarse solve
// z = (sigma M0 + S0)^-1 r on the coarsest level, in FP64 with the per-node inverse (built from the
// Cholesky factor at plan setup): the owner copies of r are gathered into LDS (one lane per system;
// read from memory instead when they do not fit), and every copy of every unknown takes its row of
// the inverse times that vector; the four wavefronts of the block share the rows.
template <typename T, bool STAGED>
__global__ __launch_bounds__(256) void k_coarse(T *z, const T *r, const double *__restrict__ Ainv,
                                                const int *__restrict__ node, int N0, const int *__restrict__ orow,
                                                const int *__restrict__ rgid, int64_t R0, int ldb,
                                                const int *__restrict__ active) {
  extern __shared__ double sh[];  // STAGED: right-hand sides [N0][64]
  const int ct = blockIdx.x;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = ct * CT + lane;
  if (STAGED) {
    for (int i = wave; i < N0; i += 4) sh[i * CT + lane] = (double)r[(int64_t)orow[i] * ldb + col];
    __syncthreads();
  }
  const double *A = Ainv + (size_t)node[col] * N0 * N0;
  // every row of the level (each copy of an unknown) takes row g of A^-1 times the right-hand side
  for (int64_t rr = wave; rr < R0; rr += 4) {
    const int g = rgid[rr];
    if (g < 0) continue;
    double acc = 0.0;
    for (int k = 0; k < N0; ++k)
      acc += A[(size_t)g * N0 + k] * (STAGED ? sh[k * CT + lane] : (double)r[(int64_t)orow[k] * ldb + col]);
    z[rr * ldb + col] = (T)acc;
  }
}

template <typename T>
void coarse_solve(const Level &C, int N0, T *z, const T *r, const double *Ainv, const int *node, int ldb,
                  int ntiles, const int *active, hipStream_t s) {
  // the right-hand sides of a column tile are staged in LDS when they fit, else read from memory
  const size_t shm = (size_t)N0 * CT * sizeof(double);
  if (shm <= 65536)
    hipLaunchKernelGGL((k_coarse<T, true>), dim3(ntiles), dim3(256), shm, s, z, r, Ainv, node, N0, C.owner_row.p,
                       C.row_gid.p, C.R, ldb, active);
  else
    hipLaunchKernelGGL((k_coarse<T, false>), dim3(ntiles), dim3(256), 0, s, z, r, Ainv, node, N0, C.owner_row.p,
                       C.row_gid.p, C.R, ldb, active);
  HIPCHK(hipGetLastError());
}
template void coarse_solve<double>(const Level &, int, double *, const double *, const double *, const int *, int,
                                   int, const int *, hipStream_t);
template void coarse_solve<float>(const Level &, int, float *, const float *, const double *, const int *, int, int,
                                  const int *, hipStream_t);

// ------------------------------------------------------------------ layout conversions
// X[row][c] = src[c][gid(row)] for c < nvec (every copy of an unknown gets its value), 0 else.
__global__ void k_g2l(double *X, const double *src, int64_t N, int nvec, const int *__restrict__ rgid, int64_t R,
                      int ldb) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (id >= R) return;
  const int g = rgid[id];
  for (int c = threadIdx.x; c < ldb; c += blockDim.x)
    X[id * ldb + c] = (g >= 0 && c < nvec) ? src[(int64_t)c * N + g] : 0.0;
}
void global_to_local(const Level &L, double *X, const double *src, int nvec, int ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_g2l, dim3((unsigned)((L.R + 3) / 4)), dim3(64, 4), 0, s, X, src, (int64_t)L.N, nvec,
                     L.row_gid.p, L.R, ldb);
  HIPCHK(hipGetLastError());
}

// dst[c][g] = X[owner_row(g)][c0 + c] for c < nvec
__global__ void k_l2g(double *dst, const double *X, int64_t N, int nvec, int c0, const int *__restrict__ orow,
                      int ldb) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (g >= N) return;
  const int64_t r = orow[g];
  for (int c = threadIdx.x; c < nvec; c += blockDim.x) dst[(int64_t)c * N + g] = X[r * ldb + c0 + c];
}
void local_to_global(const Level &L, double *dst, const double *X, int nvec, int c0, int ldb, hipStream_t s) {
  hipLaunchKernelGGL(k_l2g, dim3((unsigned)((L.N + 3) / 4)), dim3(64, 4), 0, s, dst, X, (int64_t)L.N, nvec, c0,
                     L.owner_row.p, ldb);
  HIPCHK(hipGetLastError());
}

// Y[row][k*S + s] = X[row][s]: the same right-hand side for every node
// Y[r][c] = X[r][c mod S] for c < K S, 0 for K S <= c < ncw (ncw <= ldy minus the column offset of Y)
__global__ void k_replicate(double *Y, int ldy, const double *X, int ldx, int S, int K, int ncw, int64_t R) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= R) return;
  for (int c = threadIdx.x; c < ncw; c += blockDim.x) Y[r * ldy + c] = (c < K * S) ? X[r * ldx + (c % S)] : 0.0;
}
void replicate_cols(const Level &L, double *Y, int ldy, const double *X, int ldx, int S, int K, hipStream_t s,
                    int ncw) {
  if (ncw < 0) ncw = ldy;
  hipLaunchKernelGGL(k_replicate, dim3((unsigned)((L.R + 3) / 4)), dim3(64, 4), 0, s, Y, ldy, X, ldx, S, K, ncw,
                     L.R);
  HIPCHK(hipGetLastError());
}

// Quadrature sum (eq. beta-approx): u[s][g] = sum_k omega_k X[owner(g)][k*S + s], k ascending, FP64.
__global__ void k_qsum(double *u, const double *X, const double *__restrict__ omega, int K, int S, int64_t N,
                       const int *__restrict__ orow, int ldb) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (g >= N) return;
  const int64_t r = orow[g];
  for (int s = threadIdx.x; s < S; s += blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += omega[k] * X[r * ldb + (int64_t)k * S + s];
    u[(int64_t)s * N + g] = acc;
  }
}
void quadrature_sum(const Level &L, double *u, const double *X, const double *omega, int K, int S, int ldb,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_qsum, dim3((unsigned)((L.N + 3) / 4)), dim3(64, 4), 0, s, u, X, omega, K, S, (int64_t)L.N,
                     L.owner_row.p, ldb);
  HIPCHK(hipGetLastError());
}

}  // namespace gf
