// Declarations shared by the solver kernels (k_solve.hip) and the host orchestration.
#pragma once
#include "gf_internal.h"

namespace gf {

// Per-system CG state, one entry per batch column.
struct ColState {
  double rz;     // r^T z of the current iterate
  double alpha;  // step length
  double beta;   // direction update
  double bb;     // |b|^2 (global unknowns)
  double rr;     // |r|^2 after the last update
  int done;      // 1: converged / frozen (padding columns start frozen)
  int it;        // iterations taken
  int flag;      // bit 0: max_iter reached, bit 1: breakdown
  int pad;
};

enum ReduceOp { OP_STORE = 0, OP_BB, OP_RZ0, OP_ALPHA, OP_CHECK, OP_BETA, OP_BETA_FLEX, OP_CHECK_BETA };

constexpr int kMaxRowBlocks = 1024;  // row blocks of the generic reduction kernels
constexpr int kRowBlocks = 256;      // row blocks per column tile of the streaming kernels

// partial sums [slots][ldb] and one counter per column tile
struct Scratch {
  double *partial = nullptr;
  int *counter = nullptr;
};

// Per-system scalar step applied by the last block of a column tile to the reduced sums.
__device__ inline void finalize_col(int op, int col, const double *tot, ColState *cs, double tol2, int maxit) {
  ColState &c = cs[col];
  switch (op) {
    case OP_BB:
      c.bb = tot[0];
      c.rr = tot[0];
      c.it = 0;
      c.flag = 0;
      c.alpha = 0;
      c.beta = 0;
      if (!isfinite(tot[0])) {  // a load that is not finite: CG cannot start
        c.flag |= 2;
        c.done = 1;
      } else {
        c.done = (c.done || !(tot[0] > 0.0)) ? 1 : 0;
      }
      break;
    case OP_RZ0:
      c.rz = tot[0];
      break;
    case OP_ALPHA:
      if (c.done) {
        c.alpha = 0.0;
      } else if (!(tot[0] > 0.0) || !isfinite(tot[0]) || !isfinite(c.rz)) {
        c.flag |= 2;
        c.done = 1;
        c.alpha = 0.0;
      } else {
        c.alpha = c.rz / tot[0];
      }
      break;
    case OP_CHECK:
      c.rr = tot[0];
      if (!c.done) {
        c.it += 1;
        if (!isfinite(tot[0])) {
          c.flag |= 2;
          c.done = 1;
        } else if (tot[0] <= tol2 * c.bb) {
          c.done = 1;
        } else if (c.it >= maxit) {
          c.flag |= 1;
          c.done = 1;
        }
      }
      break;
    case OP_BETA:
      c.beta = c.done ? 0.0 : tot[0] / c.rz;
      c.rz = tot[0];
      break;
    case OP_BETA_FLEX:
      // Polak-Ribiere: beta = z_new^T (r_new - r_old) / rz_old with r_new - r_old = -alpha q
      c.beta = c.done ? 0.0 : -c.alpha * tot[1] / c.rz;
      c.rz = tot[0];
      break;
    case OP_CHECK_BETA:  // tot[0] = |r|^2 (the test), tot[1] = r.z (beta), as OP_CHECK then OP_BETA
      finalize_col(OP_CHECK, col, tot, cs, tol2, maxit);
      finalize_col(OP_BETA, col, tot + 1, cs, tol2, maxit);
      break;
    default:
      break;
  }
}

// Sum of the per-block partials of one column tile, by all 256 threads of the last block: wavefront w
// adds slots w, w+4, w+8, ... (four independent chains), then the four wavefront sums are added in
// order.  The partition depends only on nslot, so the result is bitwise reproducible.
__device__ inline double sum_partials(const double *partial, int nslot, int ldb, int col) {
  __shared__ double red_sp[4][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = w;
  for (; b + 12 < nslot; b += 16) {
    s0 += partial[(int64_t)b * ldb + col];
    s1 += partial[(int64_t)(b + 4) * ldb + col];
    s2 += partial[(int64_t)(b + 8) * ldb + col];
    s3 += partial[(int64_t)(b + 12) * ldb + col];
  }
  for (; b < nslot; b += 4) s0 += partial[(int64_t)b * ldb + col];
  red_sp[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  return ((red_sp[0][lane] + red_sp[1][lane]) + red_sp[2][lane]) + red_sp[3][lane];
}

// per-system scalar step over the partials of a reduction (k_fused.hip)
void finalize(int nslot, int nd, int op, Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2,
              int maxit, double *out, hipStream_t s);

// ---- fused operator application (k_fused.hip)
enum EpiKind { EPI_STORE = 0, EPI_CHEB = 1, EPI_RESID = 2 };

template <typename T>
struct EpiArgs {
  int kind = EPI_STORE;
  // 1: accumulate x.y (STORE) or r.z_out (CHEB); 2 (CHEB, FP32 stencil path): r.z_out and z_out.q2 into
  // two sets of partial sums; the interface kernel applies `op`
  int dot = 0;
  int op = OP_STORE;
  T *y = nullptr;         // STORE: output; CHEB/RESID: patch contributions of shared rows; RESID: output
  // CHEB: new iterate, in a different buffer than the input; on entry that buffer holds the iterate
  // before the input (read when the step takes its previous direction as their difference)
  T *zout = nullptr;
  const T *r = nullptr;   // CHEB/RESID: right-hand side
  const T *dM = nullptr, *dS = nullptr, *sig = nullptr;
  // CHEB: per-system recurrence coefficients of this step, z_out = z + cf1 d + cf2 (r - A z)/D with the
  // previous direction d = z - z_prev (cf2 includes the reciprocal of the upper spectral bound)
  const T *cf1 = nullptr, *cf2 = nullptr;
  const double *q2 = nullptr;  // CHEB with dot 2: the second vector of z_out.q2
  // CHEB: bit 0 -- the previous direction equals the input iterate (first step after a start from
  // zero: z_prev = 0, zout is not read); bit 2 -- the step has a previous direction (every step but
  // the first of a sweep; cf1 and z_prev are read only then)
  int dflags = 0;
  // the largest number of distinct (ca, cb) pairs in one 64-column tile, as the caller knows it
  // (0: unknown); the combined-stencil kernel applies one stencil per pair when they fit its slots
  int nslot = 0;
  // 1: (ca, cb) is the same within every aligned group of 16 columns (the combined stencil can be
  // broadcast within 16-lane rows)
  int rows16 = 0;
};

struct ApplyGeom {
  int W, n1, ldb, ntiles, TY, NC, nseg, TX, nyb, nstrip, nsb, q;
  int grp;  // strip blocks of one column tile dispatched back to back (1: column tile fastest)
  int nslot2;  // first slot of the second set of partial sums (dot 2)
};

struct IfaceGeom {
  int ldb, ntiles, ngroups, ngb, nsb_apply;
  int nslot2;  // first slot of the second set of partial sums (dot 2)
};

ApplyGeom apply_geom(const Level &L, int ldb, int ntiles, int TY, int TXmax, int NC);
int partial_slots(const Level &L, int ldb, int ntiles);
bool stencil_offsets_fit(const Level &L, int ldb, int TY, int elem);
// whether the FP32 smoothing step can take the two inner products of dot 2 for every launch shape
bool stencil_dot2_fits(const Level &L, int ldb);
template <typename T>
void apply_fused(const Level &L, const T *stM, const T *stS, const T *x, const T *ca, const T *cb,
                 const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2,
                 int maxit, hipStream_t s, const ApplyTune &tune, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
template <typename T>
void iface_finish(const Level &L, const T *x, const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb,
                  int ntiles, int nsb_apply, double tol2, int maxit, hipStream_t s);
void update_xr2(const Level &L, double *x, double *r, const double *p, const double *q, Scratch &sc, int ldb,
                int ntiles, ColState *cs, int *active, double tol2, int maxit, hipStream_t s);
template <typename TZ>
void update_p2(const Level &L, double *p, const TZ *z, const ColState *cs, int ldb, int ntiles, const int *active,
               hipStream_t s);
template <typename T>
void epi_rows(const Level &L, const T *x, const EpiArgs<T> &e, Scratch &sc, ColState *cs, int *active, int ldb,
              int ntiles, double tol2, int maxit, hipStream_t s);
template <typename T, typename TR>
// (with bb: also |r|^2 over the owned unknowns into bb's partial sums, finalised as OP_BB into cs)
void cheb_first(const Level &L, const TR *r, T *r32, T *z, const T *dM, const T *dS, const T *sig,
                const T *cf2, int ldb, int ntiles, const int *active, hipStream_t s, Scratch *bb = nullptr,
                ColState *cs = nullptr);

template <typename T>
void cheb_first_cg(const Level &L, double *r, const double *q, T *r32, T *z, const T *dM, const T *dS, const T *sig,
                   const T *cf2, Scratch &sc, ColState *cs, int *active, int *active0, int ldb, int ntiles,
                   double tol2, int maxit, hipStream_t s);
// Jacobi-preconditioned CG step of the shifted mass systems: r -= alpha q, z = r / (dA ca + dB cb),
// |r|^2 and r.z into the partial sums, then the test and beta (OP_CHECK_BETA); active0 as cheb_first_cg
void jacobi_step(const Level &L, double *r, const double *q, double *z, const double *ca, const double *dA,
                 const double *cb, const double *dB, Scratch &sc, ColState *cs, int *active, int *active0, int ldb,
                 int ntiles, double tol2, int maxit, hipStream_t s);
template <typename TZ, typename TP = double>
void update_xp(const Level &L, double *x, TP *p, const TZ *z, const ColState *cs, const int *active0, int ldb,
               int ntiles, hipStream_t s);
// the mixed-precision outer operator on an FP32 search direction (see k_fused.hip)
bool outer_p32_fits(const Level &L, int ldb);
void apply_outer_p32(const Level &L, const float *p, const double *ca, const double *cb, const EpiArgs<double> &e,
                     Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2, int maxit,
                     hipStream_t s, const ApplyTune &tune, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

template <typename TA, typename TB>
void reduce_dot(const Level &L, const TA *a, const TB *b, Scratch &sc, int ldb, int ntiles, ColState *cs,
                int *active, int op, double tol2, int maxit, double *out, hipStream_t s);
template <typename TA, typename TB, typename TC>
void reduce_dot2(const Level &L, const TA *a, const TB *b, const TC *c, Scratch &sc, int ldb, int ntiles,
                 ColState *cs, int *active, int op, double tol2, int maxit, double *out, hipStream_t s);
template <typename TS, typename TD>
void convert_rows(const Level &L, const TS *a, TD *b, int ldb, int ntiles, const int *active, hipStream_t s);
void div_diag(const Level &L, double *v, const double *w, const double *sig, int ldb, int ntiles, hipStream_t s);
void div_diag2(const Level &L, double *v, const double *w, const double *ca, const double *dA, const double *cb,
               const double *dB, int ldb, int ntiles, const int *active, hipStream_t s);
template <typename T>
void diag_scale(const Level &L, T *z, const T *r, const T *sig, const T *dM, const T *dS, int ldb, int ntiles,
                const int *active, hipStream_t s);
void hash_fill(const Level &L, double *v, int ldb, int ntiles, hipStream_t s);
template <typename T>
void restrict_residual(const Level &F, const Level &C, T *rc, const T *r, const T *Az, int ldb, int ntiles,
                       const int *active, hipStream_t s);
template <typename T>
void prolong_add(const Level &F, const Level &C, T *zf, const T *zc, int ldb, int ntiles, const int *active,
                 hipStream_t s);
template <typename T>
void coarse_solve(const Level &C, int N0, T *z, const T *r, const double *Ainv, const int *node, int ldb, int ntiles,
                  const int *active, hipStream_t s);
void global_to_local(const Level &L, double *X, const double *src, int nvec, int ldb, hipStream_t s);
void local_to_global(const Level &L, double *dst, const double *X, int nvec, int c0, int ldb, hipStream_t s);
// Y[r][c] = X[r][c mod S] for c < K S and 0 up to column ncw (ncw < 0: the whole row, ldy columns);
// Y may point at a column offset within its rows when ncw keeps the writes inside them
void replicate_cols(const Level &L, double *Y, int ldy, const double *X, int ldx, int S, int K, hipStream_t s,
                    int ncw = -1);
void quadrature_sum(const Level &L, double *u, const double *X, const double *omega, int K, int S, int ldb,
                    hipStream_t s);
void launch_to_f32(const double *a, float *b, int64_t n, hipStream_t s);
void launch_white_noise(const Level &L, const double *z, int nsamp, double *ye, double *bl, int ldb, hipStream_t s);
// point evaluation Phi u (vals [nvec][npts]) and its transpose Phi^T r (out [nvec][N], every entry
// written): ptr [N+1] / ent list, per global coefficient in ascending point order, the entries
// i (p+1)^2 + a (p+1) + b of the points whose basis functions (a, b) it is; w [npts (p+1)^2] is work space
void launch_eval(const Level &L, int npts, const int *patch, const double *st, int nvec, const double *u,
                 double *vals, hipStream_t s);
void launch_eval_adjoint(const Level &L, int npts, const double *st, const int *ptr, const int *ent, double *w,
                         int nvec, const double *r, double *out, hipStream_t s);
// acc[s] += sum_k w[k] dots[k*nsamp + s];  out[s] = c acc[s]
void grad_accum(const double *dots, const double *w, int K, int nsamp, double *acc, hipStream_t s);
void grad_scale(const double *acc, int nsamp, double c, double *out, hipStream_t s);

}  // namespace gf
