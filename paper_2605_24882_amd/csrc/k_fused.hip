// Fused operator application and the streaming CG kernels.
//
// The patch operator (sigma M + S) of eq. mass / eq. stiffness is applied from its per-patch
// (2p+1)^2 stencils, and the consumer of the result runs in the same kernel (epilogue), so the
// product A z is never written to memory for unknowns inside a patch:
//   EPI_STORE  y = A x                       (optionally the inner product x . y)
//   EPI_RESID  y = r - A x                   (residual for the restriction)
//   EPI_CHEB   Chebyshev-Jacobi step on D^-1 A in three-term form: res = (r - A z)/D,
//              z_out = z + c1 (z - z_prev) + c2 res / b_max, with c1, c2 and b_max per system;
//              z_out overwrites z_prev         (optionally the inner product r . z_out)
// Unknowns on patch boundaries are shared with neighbouring patches: there the kernel stores its
// patch contribution, and the interface kernel sums the copies and runs the same epilogue.
//
// Mapping: one wavefront per strip of TY coefficient rows x TX coefficients of one patch and one
// 64-wide column tile (lane = system).  The wavefront keeps a (TY + 2p) x (2p + 1) window of the
// input in registers and moves it along the strip, loading one new column of TY + 2p values per
// step (one step ahead).  The stencil coefficients are shared by every system of the row: they
// arrive as vector loads and are broadcast to the wavefront through LDS.  Linear block ids are
// remapped so that every XCD walks a contiguous run of strips: the halo rows shared by
// neighbouring strips then hit the same L2.
#include "gf_internal.h"
#include "k_solve.h"
#include "k_stencil.h"

#include <hip/hip_ext.h>

namespace gf {

// The stencil coefficients of the current row (wavefront-uniform) are scalar loads; the window of x
// shifts by one column per step.  The epilogue kind and the inner-product flag are compile-time
// parameters, so a kernel keeps only the operands its epilogue uses live in scalar registers.
template <typename T, int P, int TY, int KIND, int DOT>
__global__ __launch_bounds__(256) void k_apply_fused(ApplyGeom g, const T *__restrict__ stM,
                                                     const T *__restrict__ stS, const T *__restrict__ x,
                                                     const T *__restrict__ ca, const T *__restrict__ cb, const T *__restrict__ cf1,
                                                     const T *__restrict__ cf2,
                                                     T *__restrict__ y, T *__restrict__ zout,
                                                     const T *__restrict__ r, const T *__restrict__ dM,
                                                     const T *__restrict__ dS, double *__restrict__ partial, const int *__restrict__ active,
                                                     int dflags) {
  constexpr int S = 2 * P + 1, WR = TY + 2 * P, SS = S * S;
  const int Lb = blockIdx.x;
  const int bl = (Lb & 7) * g.q + (Lb >> 3);
  if (bl >= g.nsb * g.ntiles) return;
  const int ct = bl % g.ntiles, sb = bl / g.ntiles;  // column tile fastest: contiguous rows in memory
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int W = g.W, n1 = g.n1;
  const int64_t ldb = g.ldb;
  const int strip = sb * 4 + wave;
  double acc = 0.0;
  if (strip < g.nstrip) {
    const int iyb = strip % g.nyb;
    const int seg = (strip / g.nyb) % g.nseg;
    const int m = strip / (g.nyb * g.nseg);
    const int iy0 = iyb * TY;
    const int x0 = seg * g.TX, x1 = min(x0 + g.TX, n1);
    const T a = ca[col], b = cb[col];
    T sg = 0, a1 = 0, a2 = 0;
    if (KIND == EPI_CHEB) {
      sg = a;  // the shift of this system
      if (dflags & 4) a1 = cf1[col];
      a2 = cf2[col];
    }
    const int64_t pbase = (int64_t)m * W * W;
    const int64_t ct0 = (int64_t)ct * CT;
    // window rows iy0 .. iy0 + TY + 2P - 1, clamped into the padded patch: a clamped row only feeds
    // outputs past the patch edge, which are not computed; the column of the next step is loaded
    // before the arithmetic of the current one
    int64_t roff[WR];
#pragma unroll
    for (int k = 0; k < WR; ++k) roff[k] = (pbase + (int64_t)min(iy0 + k, W - 1) * W) * ldb + ct0;
    T win[WR][S], nxt[WR];
#pragma unroll
    for (int k = 0; k < WR; ++k) {
#pragma unroll
      for (int c = 1; c < S; ++c) win[k][c] = (x + roff[k] + (int64_t)(x0 + c - 1) * ldb)[lane];
      nxt[k] = (x + roff[k] + (int64_t)(x0 + 2 * P) * ldb)[lane];
    }
    // The (M, S) stencil pair of an output row is fetched with vector loads (lane l holds
    // coefficient l of the concatenated pair), one output row ahead, staged in the wavefront's
    // own LDS slot as (M_i, S_i) pairs, and read back with every lane at the same address (a
    // broadcast read: one LDS instruction per tap instead of two lane reads per coefficient on
    // the vector ALU).  Scalar loads of the same data leave a full cache round trip per cache line
    // exposed in every step.  LDS instructions of one wavefront execute in order, so the reads
    // see the stores of the same row and the next row's stores follow the reads.
    constexpr int NCO = 2 * SS, NV = (NCO + 63) / 64;
    __shared__ typename Pair<T>::type lco[4][SS];
    auto stage = [&](const T *cv) {
      T *flat = reinterpret_cast<T *>(&lco[wave][0]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int l = v * 64 + lane;
        if (l < NCO) flat[l < SS ? 2 * l : 2 * (l - SS) + 1] = cv[v];
      }
      __builtin_amdgcn_wave_barrier();
    };
    auto coef_load = [&](int64_t crow, T *cv) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int lc = min(v * 64 + lane, NCO - 1);
        cv[v] = lc < SS ? stM[crow * SS + lc] : stS[crow * SS + (lc - SS)];
      }
    };
    T cvn[NV];
    coef_load(pbase + (int64_t)(iy0 + P) * W + (x0 + P), cvn);
    for (int ix = x0; ix < x1; ++ix) {
#pragma unroll
      for (int k = 0; k < WR; ++k) {
#pragma unroll
        for (int c = 0; c < S - 1; ++c) win[k][c] = win[k][c + 1];
        win[k][S - 1] = nxt[k];
      }
      const int64_t cn = (int64_t)min(ix + 1 + 2 * P, W - 1) * ldb;
#pragma unroll
      for (int k = 0; k < WR; ++k) nxt[k] = (x + roff[k] + cn)[lane];
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        const int iy = iy0 + t;
        if (iy >= n1) break;
        const int64_t row = pbase + (int64_t)(iy + P) * W + (ix + P);
        T cv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) cv[v] = cvn[v];
        // next output row of this wavefront: row t+1 of this step, else row 0 of the next step
        coef_load((t + 1 < TY && iy + 1 < n1) ? row + W : pbase + (int64_t)(iy0 + P) * W + (min(ix + 1, x1 - 1) + P),
                  cvn);
        stage(cv);
        T am = 0, as = 0;
#pragma unroll
        for (int dy = 0; dy < S; ++dy)
#pragma unroll
          for (int dx = 0; dx < S; ++dx) {
            const auto c = lco[wave][dy * S + dx];
            am = fma(c.x, win[t + dy][dx], am);
            as = fma(c.y, win[t + dy][dx], as);
          }
        __builtin_amdgcn_wave_barrier();
        const T Az = a * am + b * as;
        const int64_t i = row * ldb + col;
        const bool shared = (ix == 0) | (ix == n1 - 1) | (iy == 0) | (iy == n1 - 1);
        if (shared) {
          y[i] = Az;  // patch contribution; the interface kernel completes it
        } else if (KIND == EPI_STORE) {
          y[i] = Az;
          if (DOT) acc += (double)win[t + P][P] * (double)Az;
        } else if (KIND == EPI_RESID) {
          y[i] = r[i] - Az;
        } else {
          const T rv = r[i];
          const T D = sg * dM[row] + dS[row];
          const T zc = win[t + P][P];
          const T dp = (dflags & 4) ? ((dflags & 1) ? zc : zc - zout[i]) : T(0);
          const T dn = a1 * dp + a2 * ((rv - Az) / D);
          const T zo = zc + dn;
          zout[i] = zo;
          if (DOT) acc += (double)rv * (double)zo;
        }
      }
    }
  }
  if (DOT) block_partial(acc, partial, sb, (int)ldb, col);
}

// Interface completion: sum the patch contributions of every shared unknown and run the epilogue on
// each copy.  With e.dot the last block of a column tile adds the partials of both kernels (apply
// blocks first, then interface blocks, in block order) and applies the per-system step e.op.
template <typename T, typename XT = T>
__global__ __launch_bounds__(256) void k_iface_finish(IfaceGeom g, const XT *__restrict__ x, EpiArgs<T> e,
                                                      double *partial, ColState *cs,
                                                      const int *__restrict__ gp, const int *__restrict__ gr,
                                                      int *active, double tol2, int maxit) {
  const int ct = blockIdx.x % g.ntiles, gb = blockIdx.x / g.ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const int grp = gb * 4 + wave;
  double acc = 0.0, acc2 = 0.0;
  if (grp < g.ngroups) {
    const int k0 = gp[grp], k1 = gp[grp + 1];
    T s = 0;
    for (int k = k0; k < k1; ++k) s += e.y[(int64_t)gr[k] * ldb + col];
    for (int k = k0; k < k1; ++k) {
      const int64_t row = gr[k];
      const int64_t i = row * ldb + col;
      const bool own = (k == k0);
      double a2 = 0.0, a3 = 0.0;
      if (e.kind == EPI_STORE) {
        e.y[i] = s;
        if (e.dot) a2 = (double)x[i] * (double)s;
      } else if (e.kind == EPI_RESID) {
        e.y[i] = e.r[i] - s;
      } else {
        const T rv = e.r[i];
        const T D = e.sig[col] * e.dM[row] + e.dS[row];
        const T res = (rv - s) / D;
        const T zc = (T)x[i];
        const T dp = (e.dflags & 4) ? ((e.dflags & 1) ? zc : zc - e.zout[i]) : T(0);
        const T dn = ((e.dflags & 4) ? e.cf1[col] : T(0)) * dp + e.cf2[col] * res;
        const T zo = zc + dn;
        e.zout[i] = zo;
        if (e.dot) a2 = (double)rv * (double)zo;
        if (e.dot == 2) a3 = (double)zo * e.q2[i];
      }
      if (own) {
        acc += a2;
        acc2 += a3;
      }
    }
  }
  if (e.dot == 2)
    block_partial2(acc, acc2, partial, g.nsb_apply + gb, (int64_t)g.nslot2 + g.nsb_apply + gb, ldb, col);
  else if (e.dot)
    block_partial(acc, partial, g.nsb_apply + gb, ldb, col);
}

// Per-system scalar step after a reduction: one block per column tile sums the partials of all blocks
// (fixed order, see sum_partials) and applies `op`; for OP_CHECK it also refreshes the tile's
// active flag.  A separate launch rather than a last-block-done counter: the kernel boundary makes
// the partials of every block visible without device-scope fences in the producers.
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partial, int nslot, int nd, int ldb,
                                                  int op, ColState *cs, int *active, double tol2, int maxit,
                                                  double *out) {
  const int ct = blockIdx.x;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int col = ct * CT + lane;
  double tot[2] = {0.0, 0.0};
  tot[0] = sum_partials(partial, nslot, ldb, col);
  if (nd > 1) {
    __syncthreads();
    tot[1] = sum_partials(partial + (int64_t)nslot * ldb, nslot, ldb, col);
  }
  if (threadIdx.x >= 64) return;
  if (op == OP_STORE) {
    out[col] = tot[0];
    out[ldb + col] = tot[1];
    return;
  }
  finalize_col(op, col, tot, cs, tol2, maxit);
  if ((op == OP_CHECK || op == OP_CHECK_BETA) && active) {
    const unsigned long long any = __ballot(!cs[col].done);
    if (lane == 0) active[ct] = any ? 1 : 0;
  }
}

void finalize(int nslot, int nd, int op, Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2,
              int maxit, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(ntiles), dim3(256), 0, s, sc.partial, nslot, nd, ldb, op, cs, active, tol2, maxit,
                     out);
  HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ launchers
static int xcd_q(int total) { return (total + 7) / 8; }

template <typename T, int P, int TY, int KIND, int DOT>
static void launch_apply_k(const ApplyGeom &g, int algo, const T *stM, const T *stS, const T *x, const T *ca,
                           const T *cb, const EpiArgs<T> &e, double *partial, const int *active, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
  // with events the runtime stamps them at the start and end of this dispatch itself
  if (algo == 1) {
    auto kern = e.rows16 ? k_stencil<T, P, TY, KIND, DOT, SM_DPP>
                : (e.nslot >= 1 && e.nslot <= StencilSlots<T, P, TY>::value) ? k_stencil<T, P, TY, KIND, DOT, SM_COMB>
                                                                            : k_stencil<T, P, TY, KIND, DOT, SM_PAIR>;
    if (ev0)
      hipExtLaunchKernelGGL(kern, dim3(8 * g.q), dim3(256), 0, s, ev0, ev1, 0, g, stM, stS, x, ca, cb, e.cf1, e.cf2,
                            e.y, e.zout, e.r, partial, active, e.dflags, e.q2);
    else
      hipLaunchKernelGGL(kern, dim3(8 * g.q), dim3(256), 0, s, g, stM, stS, x, ca, cb, e.cf1, e.cf2, e.y, e.zout,
                         e.r, partial, active, e.dflags, e.q2);
    return;
  }
  if constexpr (DOT == 2) {
    fail(GF_EUNSUPPORTED, "two inner products need the combined-stencil kernel");
  } else if constexpr (TY <= 2) {
    if (ev0)
      hipExtLaunchKernelGGL((k_apply_fused<T, P, TY, KIND, DOT>), dim3(8 * g.q), dim3(256), 0, s, ev0, ev1, 0, g,
                            stM, stS, x, ca, cb, e.cf1, e.cf2, e.y, e.zout, e.r, e.dM, e.dS, partial, active,
                            e.dflags);
    else
      hipLaunchKernelGGL((k_apply_fused<T, P, TY, KIND, DOT>), dim3(8 * g.q), dim3(256), 0, s, g, stM, stS, x, ca,
                         cb, e.cf1, e.cf2, e.y, e.zout, e.r, e.dM, e.dS, partial, active, e.dflags);
  }
}

template <typename T, int P, int TY>
static void launch_apply_pt(const ApplyGeom &g, int algo, const T *stM, const T *stS, const T *x, const T *ca,
                            const T *cb, const EpiArgs<T> &e, double *partial, const int *active, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1) {
  if (e.kind == EPI_STORE) {
    if (e.dot) launch_apply_k<T, P, TY, EPI_STORE, 1>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
    else launch_apply_k<T, P, TY, EPI_STORE, 0>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
  } else if (e.kind == EPI_CHEB) {
    if (e.dot == 2) {
      if constexpr (sizeof(T) == 4)
        launch_apply_k<T, P, TY, EPI_CHEB, 2>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
      else
        fail(GF_EUNSUPPORTED, "two inner products in the smoothing step are an FP32 epilogue");
    } else if (e.dot) {
      launch_apply_k<T, P, TY, EPI_CHEB, 1>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
    } else {
      launch_apply_k<T, P, TY, EPI_CHEB, 0>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
    }
  } else {
    launch_apply_k<T, P, TY, EPI_RESID, 0>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
  }
}

// four rows per strip only for degrees up to 3 (an FP64 strip of four rows holds its window at one or
// two waves per SIMD; the tuner keeps it only where that pays), and only in the combined-stencil kernel
template <typename T, int P>
static void launch_apply_p(const ApplyGeom &g, int algo, const T *stM, const T *stS, const T *x, const T *ca,
                           const T *cb, const EpiArgs<T> &e, double *partial, const int *active, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (P <= 3) {
    if (g.TY == 2) {
      launch_apply_pt<T, P, 2>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
      return;
    }
    if (g.TY == 4) {
      launch_apply_pt<T, P, 4>(g, 1, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
      return;
    }
  }
  launch_apply_pt<T, P, 1>(g, algo, stM, stS, x, ca, cb, e, partial, active, s, ev0, ev1);
}

ApplyGeom apply_geom(const Level &L, int ldb, int ntiles, int TY, int TXmax, int NC) {
  ApplyGeom g;
  g.W = L.W;
  g.n1 = L.n1;
  g.ldb = ldb;
  g.ntiles = ntiles;
  g.TY = (L.p >= 4 || TY < 2) ? 1 : (TY < 4 ? 2 : 4);
  g.NC = 1;
  g.nseg = (L.n1 + TXmax - 1) / TXmax;
  g.TX = (L.n1 + g.nseg - 1) / g.nseg;
  g.nyb = (L.n1 + g.TY - 1) / g.TY;
  g.nstrip = L.npatch * g.nseg * g.nyb;
  g.nsb = (g.nstrip + 3) / 4;
  g.q = xcd_q(g.nsb * ntiles);
  g.grp = 1;
  return g;
}

// The combined-stencil kernel reads and writes through buffer descriptors based at the first row of
// its strip, with 32-bit offsets below 2^31 bytes: the window (TY + 2p rows of the padded patch and one
// more row of columns), the output rows and the stencils of the strip must fit that range.
bool stencil_offsets_fit(const Level &L, int ldb, int TY, int elem) {
  const int64_t lim = ((int64_t)1 << 31) - 1;
  const int64_t win = (int64_t)(TY + 2 * L.p + 1) * L.W * ldb * elem;
  const int64_t st = (int64_t)(TY + 1) * L.W * L.S * L.S * elem;
  return win < lim && st < lim;
}

bool stencil_dot2_fits(const Level &L, int ldb) {
  // every FP32 strip height, and the FP64 vector q2 read at output rows (TY + 1 patch rows at most)
  const int64_t lim = ((int64_t)1 << 31) - 1;
  return stencil_offsets_fit(L, ldb, 4, 4) && (int64_t)5 * L.W * ldb * 8 < lim;
}

int partial_slots(const Level &L, int ldb, int ntiles) {
  const ApplyGeom g = apply_geom(L, ldb, ntiles, 1, 16, 1);  // the most strips of any tuning candidate
  const int ngb = (L.ngroups + 3) / 4;
  return std::max(g.nsb + ngb, kRowBlocks);
}

template <typename T>
void apply_fused(const Level &L, const T *stM, const T *stS, const T *x, const T *ca, const T *cb,
                 const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2,
                 int maxit, hipStream_t s, const ApplyTune &tune, hipEvent_t ev0, hipEvent_t ev1) {
  ApplyGeom g = apply_geom(L, ldb, ntiles, tune.TY, tune.TX, tune.NC);
  g.grp = std::max(1, std::min(tune.grp, g.nsb));
  int algo = tune.algo;
  if (algo == 1 && !stencil_offsets_fit(L, ldb, g.TY, (int)sizeof(T))) {
    // the combined-stencil kernel addresses vectors by 32-bit offsets from the strip's first row
    algo = 0;
    g = apply_geom(L, ldb, ntiles, std::min(g.TY, 2), tune.TX, tune.NC);
  }
  // dot 2: the second set of partial sums follows the first (strip blocks, then interface blocks)
  g.nslot2 = g.nsb + (L.ngroups + 3) / 4;
  if (e.dot == 2 && (algo != 1 || !stencil_dot2_fits(L, ldb)))
    fail(GF_EUNSUPPORTED, "two inner products in the smoothing step need the combined-stencil kernel");
  switch (L.p) {
    case 1: launch_apply_p<T, 1>(g, algo, stM, stS, x, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 2: launch_apply_p<T, 2>(g, algo, stM, stS, x, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 3: launch_apply_p<T, 3>(g, algo, stM, stS, x, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 4: launch_apply_p<T, 4>(g, algo, stM, stS, x, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 5: launch_apply_p<T, 5>(g, algo, stM, stS, x, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    default: fail(GF_EUNSUPPORTED, "degree out of range");
  }
  HIPCHK(hipGetLastError());
  iface_finish<T>(L, x, e, sc, cs, active, ldb, ntiles, g.nsb, tol2, maxit, s);
}
template void apply_fused<double>(const Level &, const double *, const double *, const double *, const double *,
                                  const double *, const EpiArgs<double> &, Scratch &, ColState *, int *, int, int,
                                  double, int, hipStream_t, const ApplyTune &, hipEvent_t, hipEvent_t);
template void apply_fused<float>(const Level &, const float *, const float *, const float *, const float *,
                                 const float *, const EpiArgs<float> &, Scratch &, ColState *, int *, int, int, double,
                                 int, hipStream_t, const ApplyTune &, hipEvent_t, hipEvent_t);

template <typename T, typename XT>
static void iface_finish_x(const Level &L, const XT *x, const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active,
                           int ldb, int ntiles, int nsb_apply, double tol2, int maxit, hipStream_t s) {
  if (L.ngroups == 0) {
    if (e.dot) fail(GF_EUNSUPPORTED, "inner product epilogue needs interface groups");
    return;
  }
  IfaceGeom g;
  g.ldb = ldb;
  g.ntiles = ntiles;
  g.ngroups = L.ngroups;
  g.ngb = (L.ngroups + 3) / 4;
  g.nsb_apply = nsb_apply;
  g.nslot2 = nsb_apply + g.ngb;
  hipLaunchKernelGGL((k_iface_finish<T, XT>), dim3(g.ngb * ntiles), dim3(256), 0, s, g, x, e, sc.partial, cs,
                     L.grp_ptr.p, L.grp_rows.p, active, tol2, maxit);
  HIPCHK(hipGetLastError());
  if (e.dot)
    finalize(nsb_apply + g.ngb, e.dot == 2 ? 2 : 1, e.op, sc, cs, active, ldb, ntiles, tol2, maxit, nullptr, s);
}

template <typename T>
void iface_finish(const Level &L, const T *x, const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb,
                  int ntiles, int nsb_apply, double tol2, int maxit, hipStream_t s) {
  iface_finish_x<T, T>(L, x, e, sc, cs, active, ldb, ntiles, nsb_apply, tol2, maxit, s);
}

// The outer CG operator of the mixed-precision solver, q = (ca M + cb S) p with p.q, on a search
// direction stored in FP32 (FP64 stencils, arithmetic and output; each p value is widened when
// loaded).  Shift-per-16-columns tiles (DPP mode) on the combined-stencil kernel only.
template <int P>
static void launch_outer_p32(const ApplyGeom &g, const double *stM, const double *stS, const float *p,
                             const double *ca, const double *cb, const EpiArgs<double> &e, double *partial,
                             const int *active, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  auto kern = k_stencil<double, P, 1, EPI_STORE, 1, SM_DPP, float>;
  if constexpr (P <= 3) {
    if (g.TY == 2) kern = k_stencil<double, P, 2, EPI_STORE, 1, SM_DPP, float>;
    if (g.TY == 4) kern = k_stencil<double, P, 4, EPI_STORE, 1, SM_DPP, float>;
  }
  if (ev0)
    hipExtLaunchKernelGGL(kern, dim3(8 * g.q), dim3(256), 0, s, ev0, ev1, 0, g, stM, stS, p, ca, cb, e.cf1, e.cf2,
                          e.y, e.zout, e.r, partial, active, e.dflags, e.q2);
  else
    hipLaunchKernelGGL(kern, dim3(8 * g.q), dim3(256), 0, s, g, stM, stS, p, ca, cb, e.cf1, e.cf2, e.y, e.zout, e.r,
                       partial, active, e.dflags, e.q2);
}

bool outer_p32_fits(const Level &L, int ldb) { return stencil_offsets_fit(L, ldb, 4, (int)sizeof(double)); }

void apply_outer_p32(const Level &L, const float *p, const double *ca, const double *cb, const EpiArgs<double> &e,
                     Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2, int maxit,
                     hipStream_t s, const ApplyTune &tune, hipEvent_t ev0, hipEvent_t ev1) {
  if (e.kind != EPI_STORE || e.dot != 1 || !e.rows16 || tune.algo != 1 || !outer_p32_fits(L, ldb))
    fail(GF_EUNSUPPORTED, "FP32 search direction: combined-stencil operator with p.q on 16-column shift groups");
  // four-row strips too: the window of FP32 values takes the registers of an FP64 one (each value is
  // widened when loaded), so two waves per SIMD hold it; the caller's tuner picks the strip height
  ApplyGeom g = apply_geom(L, ldb, ntiles, tune.TY, tune.TX, tune.NC);
  g.nslot2 = g.nsb + (L.ngroups + 3) / 4;
  const double *stM = L.stM.p, *stS = L.stS.p;
  switch (L.p) {
    case 1: launch_outer_p32<1>(g, stM, stS, p, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 2: launch_outer_p32<2>(g, stM, stS, p, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 3: launch_outer_p32<3>(g, stM, stS, p, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 4: launch_outer_p32<4>(g, stM, stS, p, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    case 5: launch_outer_p32<5>(g, stM, stS, p, ca, cb, e, sc.partial, active, s, ev0, ev1); break;
    default: fail(GF_EUNSUPPORTED, "degree out of range");
  }
  HIPCHK(hipGetLastError());
  iface_finish_x<double, float>(L, p, e, sc, cs, active, ldb, ntiles, g.nsb, tol2, maxit, s);
}
template void iface_finish<double>(const Level &, const double *, const EpiArgs<double> &, Scratch &, ColState *,
                                   int *, int, int, int, double, int, hipStream_t);
template void iface_finish<float>(const Level &, const float *, const EpiArgs<float> &, Scratch &, ColState *, int *,
                                  int, int, int, double, int, hipStream_t);

// ------------------------------------------------------------------ streaming row kernels
// One wavefront per row and column tile, four rows per loop step so that every wavefront keeps
// four independent loads of each operand in flight.
// Blocks are numbered with the column tile fastest, so that blocks running together touch whole
// rows of the [row][column] layout (contiguous memory).
struct RowGeom {
  int64_t R;
  int W, P, n1, ldb, nrb, ntiles;
  const uint8_t *owner;
};

static RowGeom row_geom(const Level &L, int ldb) {
  RowGeom g;
  g.ntiles = ldb / CT;
  g.R = L.R;
  g.W = L.W;
  g.P = L.p;
  g.n1 = L.n1;
  g.ldb = ldb;
  g.owner = L.owner.p;
  // row blocks per column tile: 256, or up to 1024 for a batch of fewer than eight tiles (about 2048
  // blocks in all), so that a batch of one or two tiles still keeps several wavefronts per compute
  // unit in flight
  g.nrb = std::max(kRowBlocks, std::min(kMaxRowBlocks, 2048 / std::max(1, g.ntiles)));
  const int64_t need = (L.R + 15) / 16;
  if (need < g.nrb) g.nrb = (int)std::max<int64_t>(1, need);
  return g;
}

// x += alpha p, r -= alpha q; |r|^2 over owned unknowns -> convergence test
__global__ __launch_bounds__(256) void k_update_xr(RowGeom g, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   ColState *cs, double *partial, int *active,
                                                   double tol2, int maxit) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const double al = cs[col].alpha;
  const int64_t stride = (int64_t)g.nrb * 4;
  double acc = 0.0;
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    double pv[4], qv[4], xv[4], rv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) {
        const int64_t i = row * ldb + col;
        pv[u] = p[i];
        qv[u] = q[i];
        xv[u] = x[i];
        rv[u] = r[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int64_t row = r0 + u * stride;
      const int64_t i = row * ldb + col;
      const double rn = rv[u] - al * qv[u];
      x[i] = xv[u] + al * pv[u];
      r[i] = rn;
      if (g.owner[row]) acc += rn * rn;
    }
  }
  block_partial(acc, partial, rb, ldb, col);
}

// p = z + beta p
template <typename TZ>
__global__ __launch_bounds__(256) void k_update_p(RowGeom g, double *__restrict__ p, const TZ *__restrict__ z,
                                                  const ColState *cs, const int *active) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const double be = cs[col].beta;
  const int64_t stride = (int64_t)g.nrb * 4;
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    double pv[4], zv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) {
        const int64_t i = row * ldb + col;
        pv[u] = p[i];
        zv[u] = (double)z[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[u]) p[(r0 + u * stride) * ldb + col] = zv[u] + be * pv[u];
  }
}

// First Chebyshev step from z = 0: z = cf2 r / D (cf2 = c2 / b_max per system).  TR is the type of the incoming
// right-hand side; with r32 != null it is also stored in the V-cycle precision.
template <typename T, typename TR>
__global__ __launch_bounds__(256) void k_cheb_first(RowGeom g, const TR *__restrict__ r, T *__restrict__ r32,
                                                    T *__restrict__ z, const T *__restrict__ dM,
                                                    const T *__restrict__ dS, const T *__restrict__ sig,
                                                    const T *__restrict__ cf2, const int *active,
                                                    double *partial) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const T sg = sig[col], sc = cf2[col];
  const int64_t stride = (int64_t)g.nrb * 4;
  double acc = 0.0;  // with partial: |r|^2 over the owned unknowns, in the input's precision
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    TR rd[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) rd[u] = r[row * ldb + col];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int64_t row = r0 + u * stride;
      const int64_t i = row * ldb + col;
      const T rv = (T)rd[u];
      const T v = sc * rv / (sg * dM[row] + dS[row]);
      if (r32) r32[i] = rv;
      z[i] = v;
      if (partial && g.owner[row]) acc += (double)rd[u] * (double)rd[u];
    }
  }
  if (partial) block_partial(acc, partial, rb, ldb, col);
}

// The outer CG's residual update fused with the first Chebyshev step of the finest level: r -= alpha q
// in FP64 with |r|^2 over the owned unknowns into the partial sums of the convergence test (the same
// rows in the same order as k_update_xr), then the step of k_cheb_first on the new residual.  The
// iterate's update x += alpha p is left to k_update_xp, which runs over the column tiles that were
// active when the iteration began (active0, written here) -- a tile that converges in this test
// still receives its last step.
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_first_cg(RowGeom g, double *__restrict__ r, const double *__restrict__ q,
                                                       T *__restrict__ r32, T *__restrict__ z,
                                                       const T *__restrict__ dM, const T *__restrict__ dS,
                                                       const T *__restrict__ sig, const T *__restrict__ cf2,
                                                       const ColState *cs, double *partial, const int *active,
                                                       int *active0) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  const bool on = !active || active[ct];
  if (rb == 0 && threadIdx.x == 0) active0[ct] = on ? 1 : 0;
  if (!on) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const double al = cs[col].alpha;
  const T sg = sig[col], sc = cf2[col];
  const int64_t stride = (int64_t)g.nrb * 4;
  double acc = 0.0;
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    double rv[4], qv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) {
        const int64_t i = row * ldb + col;
        rv[u] = r[i];
        qv[u] = q[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int64_t row = r0 + u * stride;
      const int64_t i = row * ldb + col;
      const double rn = rv[u] - al * qv[u];
      r[i] = rn;
      if (g.owner[row]) acc += rn * rn;
      const T rt = (T)rn;
      if (r32) r32[i] = rt;
      z[i] = sc * rt / (sg * dM[row] + dS[row]);
    }
  }
  block_partial(acc, partial, rb, ldb, col);
}

// Jacobi-preconditioned CG of the shifted mass systems, one pass per iteration besides the operator:
// r -= alpha q, z = r / D with D = ca dA + cb dB per column and row, |r|^2 and r.z over the owned
// unknowns into two sets of partial sums (slots rb and nrb + rb).
__global__ __launch_bounds__(256) void k_jacobi_step(RowGeom g, double *__restrict__ r, const double *__restrict__ q,
                                                     double *__restrict__ z, const double *__restrict__ ca,
                                                     const double *__restrict__ dA, const double *__restrict__ cb,
                                                     const double *__restrict__ dB, const ColState *cs,
                                                     double *partial, const int *active, int *active0) {
  __shared__ double red2[2][4][CT];
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  const bool on = !active || active[ct];
  if (rb == 0 && threadIdx.x == 0) active0[ct] = on ? 1 : 0;
  if (!on) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const double al = cs[col].alpha, a = ca[col], b = cb[col];
  const int64_t stride = (int64_t)g.nrb * 4;
  double acc = 0.0, acc2 = 0.0;
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    double rv[4], qv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) {
        const int64_t i = row * ldb + col;
        rv[u] = r[i];
        qv[u] = q[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int64_t row = r0 + u * stride;
      const int64_t i = row * ldb + col;
      const double rn = rv[u] - al * qv[u];
      const double zn = rn / (a * dA[row] + b * dB[row]);
      r[i] = rn;
      z[i] = zn;
      if (g.owner[row]) {
        acc += rn * rn;
        acc2 += rn * zn;
      }
    }
  }
  red2[0][wave][lane] = acc;
  red2[1][wave][lane] = acc2;
  __syncthreads();
  if (wave == 0)
    for (int k = 0; k < 2; ++k)
      partial[((int64_t)k * g.nrb + rb) * ldb + col] =
          red2[k][0][lane] + red2[k][1][lane] + red2[k][2][lane] + red2[k][3][lane];
}

void jacobi_step(const Level &L, double *r, const double *q, double *z, const double *ca, const double *dA,
                 const double *cb, const double *dB, Scratch &sc, ColState *cs, int *active, int *active0, int ldb,
                 int ntiles, double tol2, int maxit, hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL(k_jacobi_step, dim3(g.nrb * ntiles), dim3(256), 0, s, g, r, q, z, ca, dA, cb, dB, cs,
                     sc.partial, active, active0);
  HIPCHK(hipGetLastError());
  finalize(g.nrb, 2, OP_CHECK_BETA, sc, cs, active, ldb, ntiles, tol2, maxit, nullptr, s);
}

// x += alpha p, p = z + beta p over the column tiles active when the iteration began (p stored as TP)
template <typename TZ, typename TP>
__global__ __launch_bounds__(256) void k_update_xp(RowGeom g, double *__restrict__ x, TP *__restrict__ p,
                                                   const TZ *__restrict__ z, const ColState *cs,
                                                   const int *active0) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  if (!active0[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const double al = cs[col].alpha, be = cs[col].beta;
  const int64_t stride = (int64_t)g.nrb * 4;
  for (int64_t r0 = (int64_t)rb * 4 + wave; r0 < g.R; r0 += 4 * stride) {
    double pv[4], xv[4], zv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + u * stride;
      ok[u] = row < g.R;
      if (ok[u]) {
        const int64_t i = row * ldb + col;
        pv[u] = (double)p[i];
        xv[u] = x[i];
        zv[u] = (double)z[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!ok[u]) continue;
      const int64_t i = (r0 + u * stride) * ldb + col;
      x[i] = xv[u] + al * pv[u];
      p[i] = (TP)(zv[u] + be * pv[u]);
    }
  }
}

template <typename T>
void cheb_first_cg(const Level &L, double *r, const double *q, T *r32, T *z, const T *dM, const T *dS, const T *sig,
                   const T *cf2, Scratch &sc, ColState *cs, int *active, int *active0, int ldb, int ntiles,
                   double tol2, int maxit, hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL(k_cheb_first_cg<T>, dim3(g.nrb * ntiles), dim3(256), 0, s, g, r, q, r32, z, dM, dS, sig, cf2,
                     cs, sc.partial, active, active0);
  HIPCHK(hipGetLastError());
  finalize(g.nrb, 1, OP_CHECK, sc, cs, active, ldb, ntiles, tol2, maxit, nullptr, s);
}
template void cheb_first_cg<double>(const Level &, double *, const double *, double *, double *, const double *,
                                    const double *, const double *, const double *, Scratch &, ColState *, int *,
                                    int *, int, int, double, int, hipStream_t);
template void cheb_first_cg<float>(const Level &, double *, const double *, float *, float *, const float *,
                                   const float *, const float *, const float *, Scratch &, ColState *, int *, int *,
                                   int, int, double, int, hipStream_t);

template <typename TZ, typename TP>
void update_xp(const Level &L, double *x, TP *p, const TZ *z, const ColState *cs, const int *active0, int ldb,
               int ntiles, hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL((k_update_xp<TZ, TP>), dim3(g.nrb * ntiles), dim3(256), 0, s, g, x, p, z, cs, active0);
  HIPCHK(hipGetLastError());
}
template void update_xp<double, double>(const Level &, double *, double *, const double *, const ColState *,
                                        const int *, int, int, hipStream_t);
template void update_xp<float, double>(const Level &, double *, double *, const float *, const ColState *,
                                       const int *, int, int, hipStream_t);
template void update_xp<float, float>(const Level &, double *, float *, const float *, const ColState *, const int *,
                                      int, int, hipStream_t);

void update_xr2(const Level &L, double *x, double *r, const double *p, const double *q, Scratch &sc, int ldb,
                int ntiles, ColState *cs, int *active, double tol2, int maxit, hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL(k_update_xr, dim3(g.nrb * ntiles), dim3(256), 0, s, g, x, r, p, q, cs, sc.partial,
                     active, tol2, maxit);
  HIPCHK(hipGetLastError());
  finalize(g.nrb, 1, OP_CHECK, sc, cs, active, ldb, ntiles, tol2, maxit, nullptr, s);
}

template <typename TZ>
void update_p2(const Level &L, double *p, const TZ *z, const ColState *cs, int ldb, int ntiles, const int *active,
               hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL(k_update_p<TZ>, dim3(g.nrb * ntiles), dim3(256), 0, s, g, p, z, cs, active);
  HIPCHK(hipGetLastError());
}
template void update_p2<double>(const Level &, double *, const double *, const ColState *, int, int, const int *,
                                hipStream_t);
template void update_p2<float>(const Level &, double *, const float *, const ColState *, int, int, const int *,
                               hipStream_t);

template <typename T, typename TR>
void cheb_first(const Level &L, const TR *r, T *r32, T *z, const T *dM, const T *dS, const T *sig,
                const T *cf2, int ldb, int ntiles, const int *active, hipStream_t s, Scratch *bb, ColState *cs) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL((k_cheb_first<T, TR>), dim3(g.nrb * ntiles), dim3(256), 0, s, g, r, r32, z, dM, dS, sig,
                     cf2, active, bb ? bb->partial : nullptr);
  HIPCHK(hipGetLastError());
  // |r|^2 of the right-hand side: the reference of the convergence test
  if (bb) finalize(g.nrb, 1, OP_BB, *bb, cs, const_cast<int *>(active), ldb, ntiles, 0.0, 0, nullptr, s);
}
template void cheb_first<double, double>(const Level &, const double *, double *, double *, const double *,
                                         const double *, const double *, const double *, int, int, const int *,
                                         hipStream_t, Scratch *, ColState *);
template void cheb_first<float, float>(const Level &, const float *, float *, float *, const float *,
                                       const float *, const float *, const float *, int, int, const int *,
                                       hipStream_t, Scratch *, ColState *);
template void cheb_first<float, double>(const Level &, const double *, float *, float *, const float *,
                                        const float *, const float *, const float *, int, int, const int *,
                                        hipStream_t, Scratch *, ColState *);

}  // namespace gf

namespace gf {

// Epilogue over every row after an operator application that wrote A x into e.y (sum-factorised
// path): the same epilogues as the fused stencil kernel, for all unknowns.
template <typename T>
__global__ __launch_bounds__(256) void k_epi_rows(RowGeom g, const T *__restrict__ x, EpiArgs<T> e,
                                                  double *partial, ColState *cs, int *active,
                                                  double tol2, int maxit) {
  const int ct = blockIdx.x % g.ntiles, rb = blockIdx.x / g.ntiles;
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int ldb = g.ldb;
  const int64_t stride = (int64_t)g.nrb * 4;
  double acc = 0.0;
  for (int64_t row = (int64_t)rb * 4 + wave; row < g.R; row += stride) {
    const int64_t i = row * ldb + col;
    const T Az = e.y[i];
    double a2 = 0.0;
    if (e.kind == EPI_STORE) {
      if (e.dot) a2 = (double)x[i] * (double)Az;
    } else if (e.kind == EPI_RESID) {
      e.y[i] = e.r[i] - Az;
    } else {
      const T rv = e.r[i];
      const T D = e.sig[col] * e.dM[row] + e.dS[row];
      const T res = (rv - Az) / D;
      const T zc = x[i];
      const T dp = (e.dflags & 4) ? ((e.dflags & 1) ? zc : zc - e.zout[i]) : T(0);
      const T dn = ((e.dflags & 4) ? e.cf1[col] : T(0)) * dp + e.cf2[col] * res;
      const T zo = zc + dn;
      e.zout[i] = zo;
      if (e.dot) a2 = (double)rv * (double)zo;
    }
    if (g.owner[row]) acc += a2;
  }
  if (!e.dot) return;
  block_partial(acc, partial, rb, ldb, col);
}

template <typename T>
void epi_rows(const Level &L, const T *x, const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb,
              int ntiles, double tol2, int maxit, hipStream_t s) {
  const RowGeom g = row_geom(L, ldb);
  hipLaunchKernelGGL(k_epi_rows<T>, dim3(g.nrb * ntiles), dim3(256), 0, s, g, x, e, sc.partial, cs,
                     active, tol2, maxit);
  HIPCHK(hipGetLastError());
  if (e.dot) finalize(g.nrb, 1, e.op, sc, cs, active, ldb, ntiles, tol2, maxit, nullptr, s);
}
template void epi_rows<double>(const Level &, const double *, const EpiArgs<double> &, Scratch &, ColState *, int *,
                               int, int, double, int, hipStream_t);
template void epi_rows<float>(const Level &, const float *, const EpiArgs<float> &, Scratch &, ColState *, int *,
                              int, int, double, int, hipStream_t);

}  // namespace gf
