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

enum ReduceOp { OP_STORE = 0, OP_BB, OP_RZ0, OP_ALPHA, OP_CHECK, OP_BETA, OP_BETA_FLEX };

constexpr int kMaxRowBlocks = 1024;

// partial sums [2][kMaxRowBlocks][ldb] and one counter per column tile
struct Scratch {
  double *partial = nullptr;
  int *counter = nullptr;
};

template <typename TA, typename TB>
void reduce_dot(const Level &L, const TA *a, const TB *b, Scratch &sc, int ldb, int ntiles, ColState *cs,
                int *active, int op, double tol2, int maxit, double *out, hipStream_t s);
template <typename TA, typename TB, typename TC>
void reduce_dot2(const Level &L, const TA *a, const TB *b, const TC *c, Scratch &sc, int ldb, int ntiles,
                 ColState *cs, int *active, int op, double tol2, int maxit, double *out, hipStream_t s);
void update_xr(const Level &L, double *x, double *r, const double *p, const double *q, Scratch &sc, int ldb,
               int ntiles, ColState *cs, int *active, double tol2, int maxit, hipStream_t s);
template <typename TZ>
void update_p(const Level &L, double *p, const TZ *z, const ColState *cs, int ldb, int ntiles, const int *active,
              hipStream_t s);
template <typename TS, typename TD>
void convert_rows(const Level &L, const TS *a, TD *b, int ldb, int ntiles, const int *active, hipStream_t s);
template <typename T>
void cheb_step(const Level &L, T *z, T *d, const T *r, const T *Az, const T *dM, const T *dS, const T *sig,
               const T *invb, T c1, T c2, int first, int ldb, int ntiles, const int *active, hipStream_t s);
void div_diag(const Level &L, double *v, const double *w, const double *sig, int ldb, int ntiles, hipStream_t s);
void hash_fill(const Level &L, double *v, int ldb, int ntiles, hipStream_t s);
template <typename T>
void restrict_residual(const Level &F, const Level &C, T *rc, const T *r, const T *Az, int ldb, int ntiles,
                       const int *active, hipStream_t s);
template <typename T>
void prolong_add(const Level &F, const Level &C, T *zf, const T *zc, int ldb, int ntiles, const int *active,
                 hipStream_t s);
template <typename T>
void coarse_solve(const Level &C, int N0, T *z, const T *r, const double *Lf, const int *node, int ldb, int ntiles,
                  const int *active, hipStream_t s);
void global_to_local(const Level &L, double *X, const double *src, int nvec, int ldb, hipStream_t s);
void local_to_global(const Level &L, double *dst, const double *X, int nvec, int c0, int ldb, hipStream_t s);
void replicate_cols(const Level &L, double *Y, int ldy, const double *X, int ldx, int S, int K, hipStream_t s);
void quadrature_sum(const Level &L, double *u, const double *X, const double *omega, int K, int S, int ldb,
                    hipStream_t s);
void launch_to_f32(const double *a, float *b, int64_t n, hipStream_t s);
void launch_white_noise(const Level &L, const double *z, int nsamp, double *ye, double *bl, int ldb, hipStream_t s);

}  // namespace gf
