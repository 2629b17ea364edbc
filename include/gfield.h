/*
 * gfield — Whittle-Matern Gaussian random fields on closed surfaces by isogeometric
 * finite elements and sinc quadrature of the Balakrishnan integral, on one AMD MI355X.
 *
 * C ABI of the solver library (libgfield.so).  The operations follow Harbrecht,
 * Sonderegger and von Rickenbach, "Simulation of Gaussian random fields on surfaces
 * using the isogeometric finite element method" (arXiv 2605.24882):
 *
 *   surface      Gamma = union of patches F_m: [0,1]^2 -> Gamma_m: the six-patch sphere
 *                family, or rational tensor-product B-spline (NURBS) patches (Sec. 2.2)
 *   space        S^0_{j,p}: continuous, patchwise tensor B-splines of degree p on
 *                2^j x 2^j elements per patch                              (Sec. 2.3)
 *   matrices     M_ij = <phi_j, phi_i>, S_ij = <grad phi_j, grad phi_i>     (Sec. 3.1, eq. FEM;
 *                pulled back to the reference square, Sec. 3.2, eq. mass / eq. stiffness)
 *   load         b ~ N(0, M), the discrete white noise                      (Sec. 3.3)
 *   field        u ~ (M^-1 A)^-beta M^-1 b, A = kappa^2 M + S, by the split beta = n + beta',
 *                n integer solves and the sinc rule for beta'               (Sec. 3.4, eq. beta-approx)
 *
 * Conventions shared by all calls
 *   - Every call returns a gf_status; on failure gf_last_error() gives a message
 *     (thread-local).  No C++ exception crosses this boundary.
 *   - Handles are created and destroyed by the caller; a space keeps its geometry alive.
 *     The library keeps no caller pointer after a call returns.
 *   - `mem` says where caller arrays live: GF_HOST (host memory; the library copies) or
 *     GF_DEVICE (device memory of the context's GPU).  All work is queued on the context's
 *     HIP stream; every call returns after that work has finished.
 *   - Vectors of unknowns are float64 in the global numbering of the space, several
 *     vectors stored one after the other: array[v * N + i] is unknown i of vector v.
 *   - Global numbering: patches in order, then coefficient row iy, then column ix (ix fastest),
 *     each coefficient whose surface point has not been seen yet gets the next number.
 *   - Arguments are validated on the host before any device work: GF_EINVAL for bad sizes,
 *     null pointers, non-finite or out-of-range parameters.
 */
#ifndef GFIELD_H
#define GFIELD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GF_ABI_VERSION 2

typedef enum {
  GF_OK = 0,
  GF_EINVAL = 1,        /* invalid argument */
  GF_ENOMEM = 2,        /* device or host allocation failed */
  GF_EDEVICE = 3,       /* HIP runtime error, or no usable gfx950 device */
  GF_ENOCONV = 4,       /* some system did not reach rtol within max_iter; outputs hold the last iterate */
  GF_EBREAKDOWN = 5,    /* conjugate gradients broke down (p^T A p <= 0 or not finite) */
  GF_EUNSUPPORTED = 6   /* a valid but unsupported request */
} gf_status;

enum { GF_HOST = 0, GF_DEVICE = 1 };

/* Message of the last failure on this thread ("" if none). */
const char *gf_last_error(void);
/* GF_ABI_VERSION of the loaded library. */
int gf_abi_version(void);

typedef struct gf_context gf_context;
typedef struct gf_geometry gf_geometry;
typedef struct gf_space gf_space;
typedef struct gf_tape gf_tape;

/* One GPU and one HIP stream: the caller's hipStream_t (which must outlive the context), or the
 * device's null stream when hip_stream is NULL (torch's default stream is the null stream).
 * GF_EDEVICE if the device does not exist or is not gfx950. */
gf_status gf_context_create(int32_t device, void *hip_stream, gf_context **out);
void gf_context_destroy(gf_context *ctx);

/* Measurement support, not part of the method: the achieved rate of the vector ALU's fused
 * multiply-add on the context's device, in TFLOP/s (2 flops per multiply-add), for precision
 * GF_PREC_FP64 (float64) or GF_PREC_MIXED (float32, scalar instructions as in the library's
 * kernels).  One kernel of independent multiply-add chains with no memory traffic, timed with
 * events on the context's stream; synchronous, a few milliseconds.  *tflops is a host pointer.
 * GF_EINVAL for a null argument or an unknown precision. */
gf_status gf_probe_fma(gf_context *ctx, int32_t precision, double *tflops);

/* The closed surface as six patches (Sec. 2.2): the radial projection of the faces of the
 * cube [-1,1]^3 with a = 2s-1, b = 2t-1,
 *   patch 0: ( 1, a, b)  1: (-1, b, a)  2: ( b, 1, a)  3: ( a,-1, b)  4: ( a, b, 1)  5: ( b, a,-1),
 * xh = v/|v| and F_m = r(xh) xh with r(x, y, z) = 1 + perturb_amp sin(3x) sin(2y) cos(z):
 * perturb_amp = 0 is the unit sphere of Sec. 4.1, 0.15 the perturbed sphere of the batching workload.
 * GF_EINVAL unless perturb_amp is finite with |perturb_amp| < 1 (so that r > 0).  The geometry holds
 * no device data; ctx may be NULL. */
gf_status gf_geometry_cubesphere(gf_context *ctx, double perturb_amp, gf_geometry **out);

/* A surface given as npatch NURBS patches (Sec. 2.2, Def. of the geometry: each patch a rational
 * tensor-product B-spline map F_m(s, t) = sum_ab N_a(s) N_b(t) w_ab X_ab / sum_ab N_a(s) N_b(t) w_ab
 * of degrees (deg_u, deg_v), 1..4).  Per patch m: ncoef[2m], ncoef[2m+1] control points along s and
 * t (degree+1 .. 4096); knots holds, patch after patch, the open knot vector along s
 * (ncoef[2m] + deg_u + 1 values) and then along t (ncoef[2m+1] + deg_v + 1 values), each with
 * deg+1 zeros, non-decreasing interior knots in (0, 1) of multiplicity at most deg, and deg+1
 * ones; ctrl holds, patch after patch, [ncoef[2m+1]][ncoef[2m]][4] = (x, y, z, weight), weights
 * positive.  Host arrays, copied; the geometry holds no device data (ctx may be NULL).  Patches
 * meet conformingly: an edge shared by two patches has the same control
 * points, weights and knots on both sides, in the same or the reverse order (relative tolerance
 * 1e-12 of the largest coordinate); the finite element space is glued (C^0) across such edges,
 * and any number of patches may share a corner.  An edge matched by no other edge is a boundary
 * (natural boundary condition).  GF_EINVAL for malformed input or an edge shared by more than two
 * patches, GF_EUNSUPPORTED for an edge collapsed to a point.  1 <= npatch <= 4096. */
gf_status gf_geometry_nurbs(gf_context *ctx, int32_t npatch, int32_t deg_u, int32_t deg_v, const int32_t *ncoef,
                            const double *knots, const double *ctrl, gf_geometry **out);
/* Number of patches of a geometry (-1 for NULL). */
int32_t gf_geometry_npatch(const gf_geometry *geom);
void gf_geometry_destroy(gf_geometry *geom);

/* Patch index and parameters of points.  Sphere family: the radial inverse of the maps above
 * (the coordinate of largest modulus picks the face).  NURBS geometries: the closest point of the
 * surface (every patch sampled on a 17 x 17 parameter grid, the promising patches refined by
 * Gauss-Newton steps on |F_m(s, t) - x|^2 within [0, 1]^2; the lower patch index on ties, as on
 * shared edges).  xyz[npts][3], patch[npts], st[npts][2], host arrays; host work only. */
gf_status gf_locate(const gf_geometry *geom, int32_t npts, const double *xyz, int32_t *patch, double *st);

/* S^0_{level,degree} on the geometry (Sec. 2.3): 1 <= degree <= 5, 0 <= level <= 12.
 * nquad: Gauss-Legendre points per direction and element for every integral of the space (Sec. 3.2
 * leaves the quadrature open): 0 selects degree + 1; degree + 1 and degree + 2 are supported (a
 * larger value gives GF_EUNSUPPORTED, a smaller non-zero one GF_EINVAL).
 * mg_levels: levels of the multigrid hierarchy, the finest being `level` (0: all levels down to 0;
 * 1 <= mg_levels <= level + 1 otherwise; the coarsest level is solved densely).
 * Builds the metric terms m = w a, G = w a K^-1 at the nquad^2 Gauss points of every element
 * (Sec. 3.2), the patch operators and the level hierarchy.  GF_EINVAL out of range. */
gf_status gf_space_create(gf_context *ctx, const gf_geometry *geom, int32_t degree, int32_t level, int32_t nquad,
                          int32_t mg_levels, gf_space **out);
void gf_space_destroy(gf_space *space);
/* Number N of unique unknowns: 6(n-2)^2 + 12(n-2) + 8 with n = 2^level + degree on the sphere
 * family; on NURBS geometries the count the gluing gives (a closed surface of P quadrilateral
 * patches with V corners and E shared edges: P(n-2)^2 + E(n-2) + V). */
int64_t gf_space_ndofs(const gf_space *space);
/* Length of one white-noise vector z for gf_white_noise: npatch * 4^level * (degree+1)^2. */
int64_t gf_space_noise_length(const gf_space *space);
/* Global number of each patch coefficient: local_to_global[(m*n + iy)*n + ix], n = 2^level + degree,
 * host array of npatch n^2 entries. */
gf_status gf_space_dofmap(const gf_space *space, int32_t *local_to_global);

/* Operator kinds of gf_space_apply. */
enum { GF_APPLY_STENCIL = 0, GF_APPLY_SUMFACT = 1 };
/* y = (sigma M + s_scale S) x for nvec vectors (eq. FEM, Sec. 3.2).  kind GF_APPLY_SUMFACT evaluates
 * the element integrals at the quadrature points on the fly (matrix-free, sum-factorised);
 * GF_APPLY_STENCIL uses the per-patch (2p+1)^2 coefficient stencils assembled from the same
 * integrals at space creation.  x, y: [nvec][N]. */
gf_status gf_space_apply(const gf_space *space, double sigma, double s_scale, int32_t nvec, const double *x,
                         double *y, int32_t mem, int32_t kind);

/* Directions of gf_space_transfer. */
enum { GF_PROLONG = 0, GF_RESTRICT = 1 };
/* Transfer between two consecutive levels of the space's multigrid hierarchy: the spline spaces are
 * nested (Sec. 2.3: the knots of level j-1 are a subset of those of level j), so every spline of level
 * j-1 is exactly a spline of level j, with coefficients P x (knot insertion, tensor product per patch).
 * level: the finer level j of the pair, lc+1 <= j <= the space's level, where lc is the coarsest level of
 * the hierarchy (the space's level + 1 - mg_levels; 0 with mg_levels = 0).
 * GF_PROLONG: y = P x, x of the coarse level [nvec][N(j-1)], y [nvec][N(j)].
 * GF_RESTRICT: y = P^T x, x [nvec][N(j)], y [nvec][N(j-1)] (the transpose the multigrid cycle applies to
 * residuals).  Unknown counts N(j) as gf_space_ndofs gives for a space of level j.  mem: GF_HOST or
 * GF_DEVICE for x and y; GF_EINVAL for a level outside the hierarchy or an unknown direction. */
gf_status gf_space_transfer(const gf_space *space, int32_t level, int32_t direction, int32_t nvec, const double *x,
                            double *y, int32_t mem);

/* What the space keeps cached for later calls: multigrid plans (one per list of shifts: per-level
 * spectral bounds and the dense coarse inverses of every node, Sec. 3.5) and workspaces (batch vectors,
 * one per batch width, precision and use).  Both caches are bounded (1 GiB of coarse inverses, 96 GiB of
 * workspaces per space; the environment variables GF_PLAN_CACHE_MB and GF_WORKSPACE_CACHE_MB set
 * others): at the start of every call that uses the space, the least recently used entries are
 * released until each fits its bound.  Any output pointer may be null.  Host memory only; GF_EINVAL
 * for a null space. */
gf_status gf_space_cache_info(const gf_space *space, int32_t *nplans, int64_t *plan_bytes, int32_t *nworkspaces,
                              int64_t *workspace_bytes);

/* gf_space_apply for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  The same operator, y = (sigma M + s_scale S) x
 * for nvec vectors (kind GF_APPLY_STENCIL or GF_APPLY_SUMFACT), on device arrays x, y ([nvec][N], on
 * the space's device); no host staging.  The patch-local work vectors live in a per-device static work
 * space of 256 MiB that the library reserves when it is loaded on a device (registered by
 * gf_context_create): GF_EINVAL when 2 R L + 2 L doubles exceed it, R the padded patch rows of the
 * space (npatch (2^level + 3 degree)^2) and L = nvec rounded up to a multiple of 64.  The stencil kind
 * runs with a fixed launch shape (no tuning pass).  The call returns once the work is queued on the
 * context's stream (it does not synchronise, so it may be captured); calls that overlap on one GPU
 * share the work space and race. */
gf_status gf_space_apply_noalloc(const gf_space *space, double sigma, double s_scale, int32_t nvec,
                                 const double *x, double *y, int32_t kind);

/* Discrete white noise b = sum_e R_e^T L_e z_e with M_e = L_e L_e^T the lower Cholesky factor of the
 * element mass matrix, so that b ~ N(0, M) when z ~ N(0, I) (Sec. 3.3).  z: [nsamp][noise_length],
 * elements in the order patch, ey, ex (ex fastest), each block of (p+1)^2 entries in element-local
 * order (b, a) with a (along s) fastest.  b: [nsamp][N]. */
gf_status gf_white_noise(const gf_space *space, int32_t nsamp, const double *z, double *b, int32_t mem);

/* Sinc rule of eq. (beta-approx) with step h and nodes y_k = k h, k = -k_minus..k_plus:
 * t_k = exp(-2 y_k), shifted systems (t_k M + kappa^2 M + S) x_k = r, weights
 * omega_k = (2 h sin(pi beta')/pi) t_k^(1-beta').  The paper's rule is h = 1/sqrt(K),
 * k_minus = k_plus = K.
 * split: GF_SPLIT_PLAIN, beta = n + beta' with n = floor(beta), one application of the rule for
 * beta'; or GF_SPLIT_IMPROVED, the modification of Sec. 3.4 for beta' near an integer: beta' < 1/3
 * (with n >= 1) gives n-1 integer solves and the rule for beta'' = (beta'+1)/2 applied twice,
 * beta' > 2/3 gives n integer solves and the rule for beta'' = beta'/2 applied twice (the second
 * application on M times the first result); otherwise the plain split. */
enum { GF_SPLIT_PLAIN = 0, GF_SPLIT_IMPROVED = 1 };
typedef struct {
  double h;
  int32_t k_minus, k_plus;
  int32_t split;
} gf_quad_rule;

enum { GF_PREC_FP64 = 0, GF_PREC_MIXED = 1 };
/* Solver options.  precision GF_PREC_FP64: everything in float64.  GF_PREC_MIXED: the multigrid
 * V-cycle and its operator applications in float32; the outer CG (its operator application,
 * residuals, inner products), the coarsest-level dense solve, the metric terms and the
 * quadrature sum in float64.  rtol: stop a system when |r| <= rtol |b| (Euclidean, global unknowns).
 * cheb_degree: Chebyshev-Jacobi smoothing steps before and after the coarse correction on the finest
 * level (0: the library's choice per batch -- three when columns x unknowns exceed 5e7 and the batch
 * runs alone, where memory traffic binds; nine for smaller batches, where launch latency binds and
 * fewer iterations pay, and for the first adjoint solve of gf_grad_kappa, whose load dL/du is rough;
 * seven for the requests of gf_sample_batch solved together); the coarser levels take one (two on
 * levels of more than 50,000 patch coefficients, and on every level for loads that have passed
 * through the inverse operator to an order of 1.5 or more), at most cheb_degree.  Each system
 * smooths on [b ia, b] (b: 1.1 x a power estimate of the largest eigenvalue of D^-1 A), ia between
 * 1/8 (1/32 for five steps or more) and (m(pi)/m(0))^2 of the 1D B-spline mass symbol by the share
 * sigma dM / (sigma dM + dS) of the mass term in the diagonal; loads that have passed through the
 * inverse operator to an order of 1.5 or more keep 1/8.
 * apply_kind: GF_APPLY_STENCIL or GF_APPLY_SUMFACT for every operator application in the solver.
 * preconditioner (Sec. 3.5): GF_PRECOND_VCYCLE, the multiplicative V-cycle above, or GF_PRECOND_BPX,
 * the additive multilevel preconditioner sum_l P_l D_l^-1 P_l^T with D_l the diagonal of
 * sigma M_l + S_l on every level and the dense solve on the coarsest (no operator application
 * inside the preconditioner; more CG iterations). */
enum { GF_PRECOND_VCYCLE = 0, GF_PRECOND_BPX = 1 };
typedef struct {
  int32_t precision;
  double rtol;
  int32_t max_iter;
  int32_t cheb_degree;
  int32_t apply_kind;
  int32_t flags;
  int32_t preconditioner; /* GF_PRECOND_VCYCLE (default) or GF_PRECOND_BPX */
} gf_solve_opts;

/* Statistics of the last solve (all fields written by the library). */
typedef struct {
  int32_t n_systems;       /* shifted systems solved (chain + nodes) x samples */
  int32_t max_iters;       /* largest CG iteration count over the systems */
  double max_rel_resid;    /* largest final |r|/|b| */
  double setup_ms;         /* plan setup (Chebyshev bounds, coarse factors) of this call */
  double solve_ms;         /* device time of the solves, conversions and the quadrature sum */
  double apply_ms;         /* with GF_FLAG_TIME_APPLY: summed duration of the outer-CG operator launches */
  int32_t apply_launches;  /* with GF_FLAG_TIME_APPLY: number of those launches */
  int32_t apply_rows;      /* rows (patch coefficients, copies included) one launch processes per column */
  double apply_col_sum;    /* with GF_FLAG_TIME_APPLY: columns processed, summed over those launches */
  double apply_bytes;      /* with GF_FLAG_TIME_APPLY: algorithmic bytes of those launches (8-byte x read
                              and y written per active column and patch row, plus the two (2p+1)^2
                              FP64 stencils per row), summed */
  double smooth_ms;        /* with GF_FLAG_TIME_APPLY: summed duration of the Chebyshev smoothing launches on
                              the finest level (same batches as apply_ms) */
  int32_t smooth_launches; /* with GF_FLAG_TIME_APPLY: number of those launches */
  double smooth_bytes;     /* with GF_FLAG_TIME_APPLY: their algorithmic bytes (the batch vectors each launch
                              reads and writes -- z, r, z_out and, where the recurrence needs it, d -- per
                              column of the tiles the launch processes and patch row, plus the two
                              stencils per row), summed; the launches of the first preconditioner
                              application before the CG loop are included */
  int32_t host_syncs;      /* times the host waited for the stream inside the CG loops of the call (one per
                              replayed chunk of CG iterations, one per iteration when eager) */
} gf_solve_stats;

/* flags */
#define GF_FLAG_MASS_SHIFT 4 /* gf_solve_shifted: the operator is M + sigma I (I the identity of the global
                                 unknowns), sigma >= 0, solved by Jacobi-preconditioned CG in FP64 (the
                                 shifted mass systems of gf_sqrt_mass) */
#define GF_FLAG_NO_GRAPH 2   /* enqueue every CG iteration eagerly instead of replaying captured HIP graphs
                                 (by default chunks of four CG iterations of every batch of the call are
                                 captured as one graph, kept for later calls with the same batches) */
#define GF_FLAG_TIME_APPLY 1 /* bracket each outer-CG operator launch and each finest-level smoothing
                                 launch of the dominant batch (the sinc nodes; the integer solves when
                                 beta is an integer) with HIP events; iterations are then enqueued
                                 eagerly (no graph replay) */

/* Field samples u for loads b (Sec. 3.4): n = floor(beta) integer solves A w_1 = b, A w_i = M w_{i-1},
 * then the sinc rule applied to r = M w_n (r = b if n = 0), u = sum_k omega_k x_k summed in ascending k.
 * Each shifted system is solved by multigrid-preconditioned CG; all nodes x samples of the
 * fractional part are solved as one batch.  kappa > 0, beta > 0, nsamp >= 1.  b, u: [nsamp][N]. */
gf_status gf_sample(gf_space *space, double kappa, double beta, const gf_quad_rule *rule,
                    const gf_solve_opts *opts, int32_t nsamp, const double *b, double *u, int32_t mem,
                    gf_solve_stats *stats);

/* The batch of shifted systems itself: (sigma_i M + S) x_i = b_i for i < nsys (the systems of
 * eq. beta-approx and of the integer chain, Sec. 3.4), solved together by the batched
 * multigrid-preconditioned CG that gf_sample uses.  sigma: host array [nsys], every entry > 0 and
 * finite (S is singular on a closed surface); at most 4096 distinct values per call.  b, x: [nsys][N]
 * (b assembled, like a load).  Errors as gf_sample. */
gf_status gf_solve_shifted(gf_space *space, int32_t nsys, const double *sigma, const double *b, double *x,
                           const gf_solve_opts *opts, int32_t mem, gf_solve_stats *stats);

/* One request of gf_sample_batch: the arguments of one gf_sample call.  Spaces may differ in degree
 * and level but must belong to the context of the batch; b and u as in gf_sample, all of the same
 * memory kind. */
typedef struct {
  gf_space *space;
  double kappa, beta;
  gf_quad_rule rule;
  int32_t nsamp;
  const double *b;
  double *u;
} gf_batch_item;

/* Several gf_sample requests solved together (Sec. 3.4 for each request).  The integer solves of
 * all requests advance step by step (step i batches every request with floor(beta) >= i); then the
 * sinc-node systems of all requests (nodes x samples each) iterate together, one CG iteration of
 * every node batch captured as one HIP graph with one branch per batch.  Requests on one space with
 * the same rule and split (and no tape) share one node batch: their columns side by side, each with
 * its own shift, under one plan for the union of their shifts.  Each request's u agrees with what
 * gf_sample returns for it alone to the solver tolerance (bit for bit when it has a batch of its own
 * and the smoothing degree is given: the same kernels then run on the same columns in the same
 * order).
 * 1 <= nitems <= 4096.  Errors as gf_sample; validation of every request precedes any work.  stats
 * aggregates over all requests (n_systems summed, max_iters and max_rel_resid maxima). */
gf_status gf_sample_batch(gf_context *ctx, int32_t nitems, const gf_batch_item *items,
                          const gf_solve_opts *opts, int32_t mem, gf_solve_stats *stats);

/* ---- the load f = sqrt(M) y of Sec. 3.3, eq. (sqrt), for y ~ N(0, I) (f ~ N(0, M)).
 *
 * With bounds 0 < lo < lambda_min(M), hi > lambda_max(M) and q = 1 - lo/hi the rule is
 *   f = (2 K sqrt(lo) / (pi Khat)) M sum_{k=1..Khat} a_k (M + w_k^2 I)^-1 y,
 *   t_k = (k - 1/2) K / Khat,  w_k = sqrt(lo) sn(t_k|q)/cn(t_k|q),  a_k = dn(t_k|q)/cn(t_k|q)^2,
 * with sn, cn, dn the Jacobi elliptic functions of parameter q and K = K(q) the complete elliptic
 * integral of the first kind at that parameter (the paper prints E; the first-kind integral is what
 * the substitution behind the rule produces).  I is the identity of the global unknowns.
 *
 * gf_sqrt_mass_rule: the shifts w_k^2, weights a_k ([khat] each, host) and the prefactor c; host
 * only.  1 <= khat <= 4096. */
gf_status gf_sqrt_mass_rule(double lo, double hi, int32_t khat, double *w2, double *a, double *c);

/* f = sqrt(M) y for nsamp vectors y ([nsamp][N], global numbering): the khat x nsamp shifted mass
 * systems are solved as one batch by CG with a Jacobi preconditioner (opts: rtol, max_iter, flags;
 * precision is FP64).  lo = hi = 0: the library estimates the bounds, hi as the largest row sum of M
 * (a Gershgorin bound; M has no negative entries) and lo as half the Rayleigh quotient after eight
 * steps of inverse iteration (an estimate, not a guaranteed bound).  Errors as gf_sample. */
gf_status gf_sqrt_mass(gf_space *space, int32_t nsamp, const double *y, double *f, int32_t khat, double lo,
                       double hi, const gf_solve_opts *opts, int32_t mem, gf_solve_stats *stats);

/* ---- differentiation in kappa (Sec. 3.4 differentiated; the sinc nodes t_k and weights omega_k do
 * not depend on kappa, sigma_k = kappa^2 + t_k).
 *
 * gf_sample_tape: gf_sample that also returns a tape holding the solutions the adjoint needs (the
 * node solutions x_{k,s} of every pass of the rule and the integer-chain solutions w_{i,s}: about
 * (passes K + n) x nsamp x N doubles of device memory).  *tape is set only on GF_OK (NULL otherwise).
 * The tape refers to its space: destroy the tape before the space.  With the improved split the
 * adjoint runs the two passes backwards: the last takes dL/du, the first M times the weighted sum of
 * the last pass's adjoint solutions. */
gf_status gf_sample_tape(gf_space *space, double kappa, double beta, const gf_quad_rule *rule,
                         const gf_solve_opts *opts, int32_t nsamp, const double *b, double *u, int32_t mem,
                         gf_tape **tape, gf_solve_stats *stats);

/* Per-sample derivative dL_s/dkappa of a loss L = sum_s L_s(u_s), given g_s = dL/du_s (global
 * coefficients, [nsamp][N], the row-major layout of u).  Adjoint route, with A = kappa^2 M + S:
 *   lambda_{k,s} = (sigma_k M + S)^-1 g_s,  mu_s = sum_k omega_k lambda_{k,s},
 *   nu_n = A^-1 M mu (A^-1 g when beta is an integer), nu_{i-1} = A^-1 M nu_i,
 *   dL_s/dkappa = -2 kappa [ sum_k omega_k lambda_{k,s}^T M x_{k,s} + sum_i nu_{i,s}^T M w_{i,s} ].
 * The adjoint systems are solved by the same batched solver with the tape's options.  A tape can be
 * used any number of times.  dl_dkappa: [nsamp].  Errors as gf_sample (GF_ENOCONV / GF_EBREAKDOWN:
 * dl_dkappa holds the value from the last iterates). */
gf_status gf_grad_kappa(gf_tape *tape, const double *dl_du, double *dl_dkappa, int32_t mem,
                        gf_solve_stats *stats);
void gf_tape_destroy(gf_tape *tape);

/* Point evaluation (Sec. 2.3): the field with global coefficients u at the surface point F_m(s, t)
 * is sum over the (p+1)^2 B-splines that do not vanish there of B_iy(t) B_ix(s) u[gid(m, iy, ix)].
 * patch: [npts] in 0..npatch-1; st: [npts][2] = (s, t) in [0, 1]^2 (gf_locate gives both for points on the
 * surface); u: [nvec][N]; vals: [nvec][npts].  All arrays of the memory kind mem.  Invalid patch or
 * parameter values give GF_EINVAL before any work. */
gf_status gf_eval(const gf_space *space, int32_t npts, const int32_t *patch, const double *st, int32_t nvec,
                  const double *u, double *vals, int32_t mem);
/* Transpose of gf_eval: out = Phi^T r, r: [nvec][npts], out: [nvec][N].  Each coefficient sums the
 * contributions of the points that touch it in ascending point order (no atomics): the result is the
 * same bit for bit on every run. */
gf_status gf_eval_adjoint(const gf_space *space, int32_t npts, const int32_t *patch, const double *st,
                          int32_t nvec, const double *r, double *out, int32_t mem);

#ifdef __cplusplus
}
#endif

#endif /* GFIELD_H */
