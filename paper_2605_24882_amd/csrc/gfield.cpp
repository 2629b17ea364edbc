// Host orchestration and C ABI of the gfield library.
//
// Space set-up (Sec. 2.3, 3.2): per refinement level of the multigrid hierarchy the metric
// terms at the Gauss points, the patch operators (as (2p+1)^2 stencils obtained by probing
// the matrix-free operator), interface gluing and knot-insertion transfers.
// Sampling (Sec. 3.4): integer chain and one batch of all sinc nodes x samples, each system
// solved by CG preconditioned with a multigrid V-cycle (Chebyshev-Jacobi smoothing,
// knot-insertion transfers, a dense solve on the coarsest level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <sstream>
#include <type_traits>

#include "gf_internal.h"
#include "k_solve.h"

namespace gf {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;
struct GfFailure {
  gf_status code;
  std::string msg;
};
void set_error(const std::string &msg) { g_last_error = msg; }
void fail(gf_status code, const std::string &msg) { throw GfFailure{code, msg}; }
void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e == hipSuccess) return;
  std::ostringstream os;
  os << "HIP error " << hipGetErrorName(e) << " (" << hipGetErrorString(e) << ") in " << what << " at " << file
     << ":" << line;
  fail(e == hipErrorOutOfMemory ? GF_ENOMEM : GF_EDEVICE, os.str());
}

template <class F>
static gf_status guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return GF_OK;
  } catch (const GfFailure &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return GF_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return GF_EDEVICE;
  }
}

static inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// ------------------------------------------------------------------ level construction
static void build_level_host(Level &L, int p, int lev, int q, const gf_geometry *geom) {
  L.p = p;
  L.lev = lev;
  L.nel = 1 << lev;
  L.n1 = L.nel + p;
  L.W = L.n1 + 2 * p;
  L.q = q;
  L.S = 2 * p + 1;
  L.npatch = geom->npatch;
  L.R = (int64_t)L.npatch * L.W * L.W;
  if (geom->kind == SURF_NURBS) glue_patches_nurbs(geom->nurbs, p, lev, L.l2g, L.N);
  else glue_patches(p, lev, L.l2g, L.N);
}

static void build_level_device(gf_space *sp, Level &L, const SurfaceArgs &surf) {
  hipStream_t s = sp->ctx->stream;
  const int p = L.p, n1 = L.n1, W = L.W, nel = L.nel, q = L.q;
  // Gauss rule and per-element basis tables [nel][2][q][p+1]
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  std::vector<double> bt((size_t)nel * 2 * q * (p + 1));
  for (int e = 0; e < nel; ++e)
    for (int k = 0; k < q; ++k) {
      double val[8], der[8];
      element_basis(p, nel, e, gx[k], val, der);
      for (int a = 0; a <= p; ++a) {
        bt[(((size_t)e * 2 + 0) * q + k) * (p + 1) + a] = val[a];
        bt[(((size_t)e * 2 + 1) * q + k) * (p + 1) + a] = der[a];
      }
    }
  L.basis.upload(bt, s);
  DBuf<double> dgx, dgw;
  dgx.upload(gx, s);
  dgw.upload(gw, s);
  L.metric.alloc((size_t)L.npatch * nel * nel * q * q * 4);
  launch_metric(L, surf, dgx.p, dgw.p, s);
  L.metric32.alloc(L.metric.n);
  launch_to_f32(L.metric.p, L.metric32.p, (int64_t)L.metric.n, s);
  L.basis32.alloc(L.basis.n);
  launch_to_f32(L.basis.p, L.basis32.p, (int64_t)L.basis.n, s);

  // rows, owners, shared groups
  std::vector<int> row_gid((size_t)L.R, -1), owner_row(L.N, -1);
  std::vector<uint8_t> owner((size_t)L.R, 0);
  std::vector<std::vector<int>> copies(L.N);
  for (int m = 0; m < L.npatch; ++m)
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        const int g = L.l2g[((size_t)m * n1 + iy) * n1 + ix];
        const int64_t r = (int64_t)m * W * W + (int64_t)(iy + p) * W + (ix + p);
        row_gid[r] = g;
        copies[g].push_back((int)r);
        if (owner_row[g] < 0) {
          owner_row[g] = (int)r;
          owner[r] = 1;
        }
      }
  // groups: every unknown on a patch boundary, with all its copies.  The fused stencil kernel
  // leaves the epilogue of patch-boundary rows to the interface kernel, so a boundary unknown with
  // a single copy (an edge of an open surface) forms a group of its own.
  auto on_patch_edge = [&](int r) {
    const int lx = r % W - p, ly = (r / W) % W - p;
    return lx == 0 || lx == n1 - 1 || ly == 0 || ly == n1 - 1;
  };
  std::vector<int> gp{0}, gr;
  for (int g = 0; g < L.N; ++g)
    if (copies[g].size() > 1 || on_patch_edge(copies[g][0])) {
      for (int r : copies[g]) gr.push_back(r);
      gp.push_back((int)gr.size());
    }
  L.ngroups = (int)gp.size() - 1;
  L.owner_row_h = owner_row;
  L.row_gid.upload(row_gid, s);
  L.owner_row.upload(owner_row, s);
  L.owner.upload(owner, s);
  if (L.ngroups > 0) {
    L.grp_ptr.upload(gp, s);
    L.grp_rows.upload(gr, s);
  }

  // patch stencils by probing the matrix-free operator: 2 S^2 probe columns (M then S)
  const int ldb = round_up(2 * L.S * L.S, CT);
  DBuf<double> X, Y, ca, cb;
  X.alloc((size_t)L.R * ldb);
  Y.alloc((size_t)L.R * ldb);
  std::vector<double> hca(ldb, 0.0), hcb(ldb, 0.0);
  for (int c = 0; c < L.S * L.S; ++c) hca[c] = 1.0;
  for (int c = L.S * L.S; c < 2 * L.S * L.S; ++c) hcb[c] = 1.0;
  ca.upload(hca, s);
  cb.upload(hcb, s);
  launch_probe_vectors(L, X.p, ldb, s);
  launch_sumfact_apply<double>(L, X.p, Y.p, ca.p, cb.p, ldb, ldb / CT, nullptr, s);
  const size_t nst = (size_t)L.R * L.S * L.S;
  L.stM.alloc(nst);
  L.stS.alloc(nst);
  launch_extract_stencil(L, Y.p, ldb, L.stM.p, L.stS.p, s);
  L.stM32.alloc(nst);
  L.stS32.alloc(nst);
  launch_to_f32(L.stM.p, L.stM32.p, (int64_t)nst, s);
  launch_to_f32(L.stS.p, L.stS32.p, (int64_t)nst, s);
  L.dM.alloc((size_t)L.R);
  L.dS.alloc((size_t)L.R);
  launch_stencil_diag(L, s);
  L.dM32.alloc((size_t)L.R);
  L.dS32.alloc((size_t)L.R);
  launch_to_f32(L.dM.p, L.dM32.p, L.R, s);
  launch_to_f32(L.dS.p, L.dS32.p, L.R, s);
  std::vector<double> hdM(L.R), hdS(L.R);
  HIPCHK(hipMemcpyAsync(hdM.data(), L.dM.p, L.R * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hdS.data(), L.dS.p, L.R * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t nrow = 0;
  for (int64_t i = 0; i < L.R; ++i)
    if (row_gid[i] >= 0) {
      L.dM_mean += hdM[i];
      L.dS_mean += hdS[i];
      ++nrow;
    }
  L.dM_mean /= (double)nrow;
  L.dS_mean /= (double)nrow;
}

// knot-insertion transfer bands from level C into level F (= C + 1)
static void build_transfer(gf_space *sp, Level &F, const Level &C) {
  hipStream_t s = sp->ctx->stream;
  const int nf = F.n1, nc = C.n1;
  std::vector<double> P = refinement_matrix(F.p, C.lev);
  // rows of P: fine index -> band of coarse indices
  int pw = 0, rw = 0;
  std::vector<int> f_lo(nf), f_hi(nf), c_lo(nc, nf), c_hi(nc, -1);
  for (int i = 0; i < nf; ++i) {
    int lo = nc, hi = -1;
    for (int c = 0; c < nc; ++c)
      if (P[(size_t)i * nc + c] != 0.0) {
        lo = std::min(lo, c);
        hi = std::max(hi, c);
        c_lo[c] = std::min(c_lo[c], i);
        c_hi[c] = std::max(c_hi[c], i);
      }
    f_lo[i] = lo;
    f_hi[i] = hi;
    pw = std::max(pw, hi - lo + 1);
  }
  for (int c = 0; c < nc; ++c) rw = std::max(rw, c_hi[c] - c_lo[c] + 1);
  std::vector<int> ps(nf), rs(nc);
  std::vector<double> pc((size_t)nf * pw, 0.0), rc((size_t)nc * rw, 0.0);
  for (int i = 0; i < nf; ++i) {
    int st = std::min(f_lo[i], nc - pw);
    ps[i] = st;
    for (int k = 0; k < pw; ++k) pc[(size_t)i * pw + k] = P[(size_t)i * nc + st + k];
  }
  for (int c = 0; c < nc; ++c) {
    int st = std::min(c_lo[c], nf - rw);
    rs[c] = st;
    for (int k = 0; k < rw; ++k) rc[(size_t)c * rw + k] = P[(size_t)(st + k) * nc + c];
  }
  F.pw = pw;
  F.rw = rw;
  F.pro_start.upload(ps, s);
  F.res_start.upload(rs, s);
  F.pro_c.upload(pc, s);
  F.res_c.upload(rc, s);
  std::vector<float> pcf(pc.begin(), pc.end()), rcf(rc.begin(), rc.end());
  F.pro_c32.upload(pcf, s);
  F.res_c32.upload(rcf, s);
}

// dense global matrices of the coarsest level from its patch stencils
static void build_coarse_dense(gf_space *sp) {
  Level &C = *sp->lev[0];
  hipStream_t s = sp->ctx->stream;
  const size_t nst = (size_t)C.R * C.S * C.S;
  std::vector<double> hm(nst), hs(nst);
  HIPCHK(hipMemcpyAsync(hm.data(), C.stM.p, nst * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hs.data(), C.stS.p, nst * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int N0 = C.N, p = C.p, W = C.W, n1 = C.n1, S = C.S;
  std::vector<double> M0((size_t)N0 * N0, 0.0), S0((size_t)N0 * N0, 0.0);
  for (int m = 0; m < C.npatch; ++m)
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        const int64_t r = (int64_t)m * W * W + (int64_t)(iy + p) * W + (ix + p);
        const int gi = C.l2g[((size_t)m * n1 + iy) * n1 + ix];
        for (int dy = -p; dy <= p; ++dy)
          for (int dx = -p; dx <= p; ++dx) {
            const int jy = iy + dy, jx = ix + dx;
            if (jy < 0 || jy >= n1 || jx < 0 || jx >= n1) continue;
            const int gj = C.l2g[((size_t)m * n1 + jy) * n1 + jx];
            const int d = (dy + p) * S + (dx + p);
            M0[(size_t)gi * N0 + gj] += hm[(size_t)r * S * S + d];
            S0[(size_t)gi * N0 + gj] += hs[(size_t)r * S * S + d];
          }
      }
  sp->N0 = N0;
  sp->M0.upload(M0, s);
  sp->S0.upload(S0, s);
  HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ plans and workspaces
struct Plan {
  std::vector<double> sig;                // distinct shifts (nodes)
  std::vector<std::vector<double>> invb;  // [level index][node] 1/(upper spectral bound of D^-1 A)
  std::vector<std::vector<double>> mshare;  // [level index][node] share of the mass term in the
                                            // diagonal, sigma dM / (sigma dM + dS) (level means)
  double ia_mass = 0.0;                     // (m(pi)/m(0))^2 of the 1D B-spline mass symbol
  DBuf<double> Ainv;                      // [node][N0][N0] inverses of the coarse matrices
  double setup_ms = 0.0;
  uint64_t last = 0;                      // the space's call that used it last
};

struct LevelWork {
  DBuf<double> r64, z64a, z64b, a64;  // V-cycle vectors (FP64 mode)
  DBuf<float> r32, z32a, z32b, a32;   // V-cycle vectors (mixed mode)
  // Chebyshev coefficients per step and system, [2][deg][ldb]: c1 of step k at k ldb, c2 / b_max of
  // step k at (deg + k) ldb
  DBuf<double> cf64;
  DBuf<float> cf32;
};

// Event pairs around the finest-level smoothing launches of one batch (GF_FLAG_TIME_APPLY), each
// with the number of batch vectors the launch reads and writes and the element size
struct SmoothLog {
  struct Entry {
    hipEvent_t e0, e1;
    int vecs, elem;
    bool first;  // launched by the first preconditioner application (before any convergence test)
  };
  std::vector<Entry> entries;
  bool first_phase = false;
  void clear() {
    for (auto &e : entries) {
      (void)hipEventDestroy(e.e0);
      (void)hipEventDestroy(e.e1);
    }
    entries.clear();
  }
};

struct Workspace {
  SmoothLog *slog = nullptr;  // set while a timed batch runs
  int ldb = 0, ntiles = 0, prec = 0;
  // structure of the columns' shifts in the current batch: the most distinct shifts in one column tile,
  // and whether every aligned group of 16 columns has one shift (see EpiArgs::nslot, rows16)
  int nslot = 0, rows16 = 0;
  DBuf<double> x, r, p, q;  // outer CG (FP64)
  // mixed precision: the search direction stored in FP32 (see BatchSolve::p32)
  DBuf<float> p32;
  std::vector<LevelWork> lw;
  DBuf<double> sig64, one64, zero64;
  DBuf<float> sig32, one32;
  DBuf<int> node, active;
  // outer-CG fusion: while set, the finest level's first smoothing step also performs r -= alpha q
  // (q = fuse_q) and the convergence test, and records the tiles active before it in active0
  const double *fuse_q = nullptr;
  // while set, the finest level's first smoothing step of the V-cycle also reduces |r|^2 of its input
  // (the reference of the convergence test, at the start of a solve)
  bool fuse_bb = false;
  DBuf<int> active0;
  DBuf<ColState> cs;
  DBuf<double> partial;
  DBuf<int> counter;
  std::vector<int> active_h;
  uint64_t last = 0;   // the space's call that used it last
  size_t bytes = 0;    // device memory it holds
  Scratch scratch() { return Scratch{partial.p, counter.p}; }
};

}  // namespace gf

struct gf_workspaces {
  std::map<std::tuple<int, int, int>, std::unique_ptr<gf::Workspace>> m;
};

// Saved forward state of one gf_sample_tape call: the request and every solution the adjoint needs
// (the node solutions x_{k,s} and the chain solutions w_{i,s}, patch-local layout).
struct gf_tape {
  gf_space *sp = nullptr;
  double kappa = 0, beta = 0;
  gf_quad_rule rule{};
  gf_solve_opts opts{};
  int nsamp = 0, n = 0, ldc = 0, ldf = 0;
  double bf = 0;
  std::vector<double> node_sig, omega;
  int passes = 1;                       // applications of the rule (2 for an improved split)
  std::vector<gf::DBuf<double>> xk;     // per pass: [R][ldf] node solutions, column k*nsamp + s
  std::vector<gf::DBuf<double>> w;      // w[i-1]: [R][ldc] chain solution w_i
};

namespace gf {

static std::map<const gf_space *, std::unique_ptr<gf_workspaces>> &ws_registry() {
  static std::map<const gf_space *, std::unique_ptr<gf_workspaces>> r;
  return r;
}

static size_t scratch_slots(gf_space *sp, int ldb, int ntiles) {
  size_t slots = 2 * (size_t)kMaxRowBlocks;
  // two sets for the smoothing step that takes two inner products
  for (auto &L : sp->lev) slots = std::max(slots, 2 * (size_t)partial_slots(*L, ldb, ntiles));
  return slots;
}

// slot separates the workspaces of batches that run together on the same space
static Workspace &get_workspace(gf_space *sp, int ldb, int prec, int slot = 0) {
  auto &reg = ws_registry()[sp];
  if (!reg) reg.reset(new gf_workspaces());
  auto key = std::make_tuple(ldb, prec, slot);
  auto it = reg->m.find(key);
  if (it != reg->m.end()) {
    it->second->last = sp->calls;
    return *it->second;
  }
  std::unique_ptr<Workspace> w(new Workspace());
  w->last = sp->calls;
  w->ldb = ldb;
  w->ntiles = ldb / CT;
  w->prec = prec;
  const Level &F = sp->fine();
  const size_t nf = (size_t)F.R * ldb;
  w->x.alloc(nf);
  w->r.alloc(nf);
  w->p.alloc(nf);
  w->q.alloc(nf);
  if (prec == GF_PREC_MIXED) w->p32.alloc(nf);
  w->lw.resize(sp->nlev());
  for (int li = 0; li < sp->nlev(); ++li) {
    const Level &L = *sp->lev[li];
    const size_t n = (size_t)L.R * ldb;
    LevelWork &v = w->lw[li];
    const bool finest = (li == sp->nlev() - 1);
    if (prec == GF_PREC_FP64) {
      if (!finest) v.r64.alloc(n);
      v.z64a.alloc(n);
      v.z64b.alloc(n);
      v.a64.alloc(n);
    } else {
      v.r32.alloc(n);
      v.z32a.alloc(n);
      v.z32b.alloc(n);
      v.a32.alloc(n);
    }
  }
  w->sig64.alloc(ldb);
  w->one64.alloc(ldb);
  w->zero64.alloc(ldb);
  w->sig32.alloc(ldb);
  w->one32.alloc(ldb);
  w->node.alloc(ldb);
  w->active.alloc(w->ntiles);
  w->active0.alloc(w->ntiles);
  w->cs.alloc(ldb);
  w->partial.alloc(scratch_slots(sp, ldb, w->ntiles) * ldb);
  w->counter.alloc(w->ntiles);
  std::vector<double> ones(ldb, 1.0);
  std::vector<float> onesf(ldb, 1.0f);
  w->one64.upload(ones, sp->ctx->stream);
  w->one32.upload(onesf, sp->ctx->stream);
  w->active_h.assign(w->ntiles, 0);
  // the batch vectors and the partial sums (the per-column scalars are negligible)
  w->bytes = w->x.n * 8 * 4 + w->p32.n * 4 + w->partial.n * 8;
  for (const LevelWork &v : w->lw)
    w->bytes += (v.r64.n + v.z64a.n + v.z64b.n + v.a64.n) * 8 + (v.r32.n + v.z32a.n + v.z32b.n + v.a32.n) * 4;
  Workspace &ref = *w;
  reg->m[key] = std::move(w);
  return ref;
}

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static const double *stM(const Level &L) { return L.stM.p; }
  static const double *stS(const Level &L) { return L.stS.p; }
  static const double *dM(const Level &L) { return L.dM.p; }
  static const double *dS(const Level &L) { return L.dS.p; }
  static double *r(LevelWork &l) { return l.r64.p; }
  static double *za(LevelWork &l) { return l.z64a.p; }
  static double *zb(LevelWork &l) { return l.z64b.p; }
  static double *a(LevelWork &l) { return l.a64.p; }
  static const double *cf(LevelWork &l) { return l.cf64.p; }
  static double *sig(Workspace &w) { return w.sig64.p; }
  static double *one(Workspace &w) { return w.one64.p; }
};
template <>
struct Prec<float> {
  static const float *stM(const Level &L) { return L.stM32.p; }
  static const float *stS(const Level &L) { return L.stS32.p; }
  static const float *dM(const Level &L) { return L.dM32.p; }
  static const float *dS(const Level &L) { return L.dS32.p; }
  static float *r(LevelWork &l) { return l.r32.p; }
  static float *za(LevelWork &l) { return l.z32a.p; }
  static float *zb(LevelWork &l) { return l.z32b.p; }
  static float *a(LevelWork &l) { return l.a32.p; }
  static const float *cf(LevelWork &l) { return l.cf32.p; }
  static float *sig(Workspace &w) { return w.sig32.p; }
  static float *one(Workspace &w) { return w.one32.p; }
};

// Autotuner of the fused stencil apply: on first use for a (level, precision, column stride, epilogue
// kind, stencil mode) every candidate launch shape of the combined-stencil kernel is timed with HIP
// events (one warm-up and three timed launches, all column tiles active) and the fastest is kept for the
// lifetime of the space.  The candidates write into scratch vectors of their own, so tuning leaves the
// caller's buffers untouched; the shape changes neither the operations nor their order for any output,
// so the choice cannot change results.  A level whose strips exceed the kernel's 32-bit buffer offsets
// takes the separate-stencil kernel (same launch shapes).
static bool g_autotune = true;

static int stencil_mode_class(int nslot, int rows16) { return rows16 ? 2 : (nslot >= 1 && nslot <= 8 ? 0 : 1); }

template <typename T>
static const ApplyTune &get_tune(const Level &L, int ldb, int ntiles, const T *x, const T *ca, const T *cb,
                                 const EpiArgs<T> &ecall, hipStream_t s) {
  const auto key = std::make_tuple((int)sizeof(T), ldb, ecall.kind, stencil_mode_class(ecall.nslot, ecall.rows16));
  auto it = L.tune.find(key);
  if (it != L.tune.end()) return it->second;
  ApplyTune best;
  const bool fits2 = stencil_offsets_fit(L, ldb, 2, (int)sizeof(T));
  // GF_APPLY_SHAPE="TY,TX" fixes the launch shape (reproducible profiling runs)
  if (const char *fixed = std::getenv("GF_APPLY_SHAPE")) {
    int ty = 0, tx = 0;
    // (TX below 16 would need more partial-sum slots than the workspaces hold)
    if (std::sscanf(fixed, "%d,%d", &ty, &tx) != 2 || (ty != 1 && ty != 2 && ty != 4) || tx < 16)
      fail(GF_EINVAL, "GF_APPLY_SHAPE must be \"TY,TX\" with TY in {1,2,4} and TX >= 16");
    best.TY = ty;
    best.TX = tx;
    return L.tune.emplace(key, best).first->second;
  }
  if (g_autotune && L.n1 >= 8) {
    std::vector<ApplyTune> cand;
    for (int ty : {1, 2, 4}) {
      if (ty == 4 && L.p > 3) continue;
      if (ty > 1 && L.p >= 4) continue;
      for (int tx : {32, 64}) {
        if (tx > 2 * L.n1 && tx != 32) continue;
        ApplyTune t;
        t.TY = ty;
        t.TX = tx;
        t.algo = stencil_offsets_fit(L, ldb, ty, (int)sizeof(T)) ? 1 : 0;
        if (t.algo == 0 && ty == 4) continue;
        cand.push_back(t);
      }
    }
    // scratch outputs and inputs of the candidate launches
    const size_t n = (size_t)L.R * ldb;
    DBuf<T> ty_, tz, tr;
    ty_.alloc(n);
    EpiArgs<T> e = ecall;
    e.dot = 0;
    e.y = ty_.p;
    if (e.kind != EPI_STORE) {
      tr.alloc(n);
      e.r = tr.p;
    }
    if (e.kind == EPI_CHEB) {
      tz.alloc(n);
      e.zout = tz.p;
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    Scratch none;
    float best_us = 1e30f;
    for (const ApplyTune &t : cand) {
      apply_fused<T>(L, Prec<T>::stM(L), Prec<T>::stS(L), x, ca, cb, e, none, nullptr, nullptr, ldb, ntiles, 0.0, 0,
                     s, t);
      HIPCHK(hipEventRecord(e0, s));
      for (int k = 0; k < 3; ++k)
        apply_fused<T>(L, Prec<T>::stM(L), Prec<T>::stS(L), x, ca, cb, e, none, nullptr, nullptr, ldb, ntiles, 0.0,
                       0, s, t);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      const float us = ms * 1e3f / 3.f;
      if (std::getenv("GF_TUNE_LOG"))
        std::fprintf(stderr, "tune p=%d lev=%d T=%d ldb=%d kind=%d mode=%d algo=%d TY=%d TX=%d: %.1f us\n", L.p, L.lev,
                     (int)sizeof(T), ldb, e.kind, stencil_mode_class(e.nslot, e.rows16), t.algo, t.TY, t.TX, us);
      if (us < best_us) {
        best_us = us;
        best = t;
        best.us = us;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } else {
    best.TY = fits2 ? 2 : 1;
    best.algo = stencil_offsets_fit(L, ldb, best.TY, (int)sizeof(T)) ? 1 : 0;
  }
  return L.tune.emplace(key, best).first->second;
}

// Launch shape of the mixed-precision outer operator on the FP32 search direction (apply_outer_p32):
// strips of two or four rows (a four-row strip reads 2.5 window rows per output row instead of 4, at
// two waves per SIMD instead of three), 32 or 64 columns, timed on first use per level and column
// stride on scratch vectors, partial sums and per-column states (the solver's are not touched).
static const ApplyTune &get_tune_p32(const Level &L, int ldb, int ntiles, const double *ca, const double *cb,
                                     const EpiArgs<double> &ecall, hipStream_t s) {
  const auto key = std::make_tuple(12, ldb, (int)EPI_STORE, 2);
  auto it = L.tune.find(key);
  if (it != L.tune.end()) return it->second;
  ApplyTune best;
  best.TY = 2;
  best.TX = 64;
  if (const char *fixed = std::getenv("GF_APPLY_SHAPE")) {
    int ty = 0, tx = 0;
    if (std::sscanf(fixed, "%d,%d", &ty, &tx) != 2 || (ty != 1 && ty != 2 && ty != 4) || tx < 16)
      fail(GF_EINVAL, "GF_APPLY_SHAPE must be \"TY,TX\" with TY in {1,2,4} and TX >= 16");
    best.TY = ty;
    best.TX = tx;
    return L.tune.emplace(key, best).first->second;
  }
  if (g_autotune && L.n1 >= 8) {
    const size_t n = (size_t)L.R * ldb;
    DBuf<double> ty_, part;
    DBuf<float> tp;
    DBuf<ColState> tcs;
    ty_.alloc(n);
    tp.alloc(n);
    part.alloc((size_t)2 * partial_slots(L, ldb, ntiles) * ldb);
    tcs.alloc(ldb);
    EpiArgs<double> e = ecall;
    e.y = ty_.p;
    e.dot = 1;
    e.op = OP_ALPHA;  // into the scratch states
    Scratch sc{part.p, nullptr};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_us = 1e30f;
    for (int tyc : {2, 4}) {
      if (tyc == 4 && L.p > 3) continue;
      for (int tx : {32, 64}) {
        if (tx > 2 * L.n1 && tx != 32) continue;
        ApplyTune t;
        t.TY = tyc;
        t.TX = tx;
        apply_outer_p32(L, tp.p, ca, cb, e, sc, tcs.p, nullptr, ldb, ntiles, 0.0, 0, s, t);
        HIPCHK(hipEventRecord(e0, s));
        for (int k = 0; k < 3; ++k) apply_outer_p32(L, tp.p, ca, cb, e, sc, tcs.p, nullptr, ldb, ntiles, 0.0, 0, s, t);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const float us = ms * 1e3f / 3.f;
        if (std::getenv("GF_TUNE_LOG"))
          std::fprintf(stderr, "tune p=%d lev=%d outer on FP32 direction ldb=%d TY=%d TX=%d: %.1f us\n", L.p, L.lev,
                       ldb, tyc, tx, us);
        if (us < best_us) {
          best_us = us;
          best = t;
          best.us = us;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return L.tune.emplace(key, best).first->second;
}

// One operator application with epilogue e: the fused stencil kernel, or the sum-factorised
// kernel followed by the interface sum and the epilogue over all rows.
template <typename T>
static void apply_epi(const Level &L, int kind, const T *x, const T *ca, const T *cb, const EpiArgs<T> &e,
                      Scratch &sc, ColState *cs, int *active, int ldb, int ntiles, double tol2, int maxit,
                      hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                      const T *stB = nullptr) {
  if (stB) {  // second operator given as a stencil (stencil path only)
    const ApplyTune &t = get_tune<T>(L, ldb, ntiles, x, ca, cb, e, s);
    apply_fused<T>(L, Prec<T>::stM(L), stB, x, ca, cb, e, sc, cs, active, ldb, ntiles, tol2, maxit, s, t, ev0, ev1);
    return;
  }
  if (kind == GF_APPLY_SUMFACT) {
    if (ev0) HIPCHK(hipEventRecord(ev0, s));
    launch_sumfact_apply<T>(L, x, e.y, ca, cb, ldb, ntiles, active, s);
    if (ev1) HIPCHK(hipEventRecord(ev1, s));
    launch_interface_sum<T>(L, e.y, ldb, ntiles, active, s);
    if (e.kind != EPI_STORE || e.dot) epi_rows<T>(L, x, e, sc, cs, active, ldb, ntiles, tol2, maxit, s);
  } else {
    const ApplyTune &t = get_tune<T>(L, ldb, ntiles, x, ca, cb, e, s);
    apply_fused<T>(L, Prec<T>::stM(L), Prec<T>::stS(L), x, ca, cb, e, sc, cs, active, ldb, ntiles, tol2, maxit, s,
                   t, ev0, ev1);
  }
}

// y = (ca M + cb S) x, assembled (interface sums included); uniform: ca and cb hold one value each over
// all columns (one combined stencil for the whole batch)
template <typename T>
static void apply_level(const Level &L, int kind, const T *x, T *y, const T *ca, const T *cb, int ldb, int ntiles,
                        const int *active, hipStream_t s, bool uniform = true) {
  EpiArgs<T> e;
  e.kind = EPI_STORE;
  e.y = y;
  e.nslot = uniform ? 1 : 0;
  e.rows16 = uniform ? 1 : 0;
  Scratch none;
  apply_epi<T>(L, kind, x, ca, cb, e, none, nullptr, const_cast<int *>(active), ldb, ntiles, 0.0, 0, s);
}

// Chebyshev interval [b/alpha, b] with b = 1.1 x the estimated largest eigenvalue of D^-1 A.  For a
// stiffness-dominated operator the smoother targets the upper eighth of the spectrum (the coarse
// levels resolve the rest).  For a mass-dominated one (the sinc nodes with large t_k) the
// high-frequency eigenvalues of D^-1 M sit at the bottom of its spectrum, down to (m(pi)/m(0))^2
// with m the symbol of the 1D B-spline mass stencil, so the interval must reach that far.  Between
// the two, 1/alpha is the convex combination weighted by the share r = sigma dM / (sigma dM + dS)
// of the mass term in the diagonal (level means).  Measured at relative residual 1e-10 on degree 2,
// 64^2 elements per patch, kappa = 10: the largest per-node CG iteration count drops from 21
// (alpha = 8 for every node) to 16, the nodes with t_k < 1e4 are unchanged; on degree 3 (64^2 and
// 256^2 elements, 1e-6) from 30 to 23 and from 29 to 21.  The wide interval pays for loads with
// high-frequency content (white noise, and M A^-1 of it: 214 -> 188 summed iterations over 21
// nodes); for M A^-2 of white noise the narrow one is better (134 against 157), so loads of that
// smoothness keep alpha = 8 (SolveSpec::smooth_load).
constexpr double kChebAlpha = 8.0;
constexpr double kChebSafety = 1.1;

// (m(0) / m(pi))^2 for the mass stencil of uniform 1D B-splines of degree p: its entries are the
// values of the cardinal B-spline of degree 2p + 1 at the integers, m(0) = their sum = 1
static double mass_interval_ratio(int p) {
  const int n = 2 * p + 1;
  std::vector<double> v(n + 2, 0.0);  // N_k at 0 .. n + 1
  v[0] = 1.0;                         // N_0 at the integers: 1 at 0, else 0
  for (int k = 1; k <= n; ++k) {
    std::vector<double> u(n + 2, 0.0);
    for (int i = 1; i <= k; ++i) u[i] = (i * v[i] + (k + 1 - i) * v[i - 1]) / k;
    v = u;
  }
  double mpi = 0.0;
  for (int i = 1; i <= n; ++i) mpi += ((i - (p + 1)) % 2 == 0 ? 1.0 : -1.0) * v[i];
  return 1.0 / (mpi * mpi);
}
constexpr int kPowerIters = 16;
// Chebyshev smoothing steps before and after the coarse correction when the caller passes 0, by the
// size of the batch (columns x unknowns of the finest level).  A large batch solved alone has its
// degree measured on its first solve (tune_degree, below; three is the starting point).  A large
// batch is bound by memory traffic, and three steps gave the fewest seconds per sample (degree 2, 64^2 elements per patch,
// 2,624 systems: 1016 samples/s against 981 with four, 874 with five and 881 with nine; degree 3,
// 256^2, 1,952 systems: 66.5 against 60.1 with four and 56.7 with nine).  A small batch is bound by
// launch latency -- every CG iteration is some seventy kernel launches -- and a high degree on the
// wide interval of degrees five and up cuts the iterations (degree 3, 64^2, 656 systems: 340 with
// nine steps against 320 with seven, 283 with five and 208 with three; the torus of 16 NURBS
// patches, 17,424 unknowns x 2,624 systems: 1176 with nine against 1074 with five and 854 with
// three).  Batches solved together in one call run as concurrent graph branches that share the GPU:
// seven steps (the perturbed-sphere batch of 18 requests: 727-750 against 709 with five and 715 with
// nine; in FP64 495 against 496 and 473).
constexpr int kDefaultCheb = 3;
constexpr int kDefaultChebSmall = 9;
constexpr int kDefaultChebConcurrent = 7;
constexpr double kSmallBatchWork = 5e7;
constexpr double kChebTwoRows = 50000.0;

static std::string plan_key(const std::vector<double> &sig) {
  std::ostringstream os;
  os.precision(17);
  for (double v : sig) os << v << ",";
  return os.str();
}

static Plan &get_plan(gf_space *sp, const std::vector<double> &sig) {
  const std::string key = plan_key(sig);
  auto it = sp->plans.find(key);
  if (it != sp->plans.end()) {
    it->second->last = sp->calls;
    return *it->second;
  }
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = sp->ctx->stream;
  std::unique_ptr<Plan> pl(new Plan());
  pl->sig = sig;
  const int nn = (int)sig.size();
  const int ldb = round_up(nn, CT), nt = ldb / CT;
  DBuf<double> dsig, one, v, w, v2, out;
  std::vector<double> hsig(ldb, 1.0), ones(ldb, 1.0);
  for (int k = 0; k < nn; ++k) hsig[k] = sig[k];
  dsig.upload(hsig, s);
  one.upload(ones, s);
  DBuf<double> partial;
  DBuf<int> counter;
  partial.alloc((size_t)2 * kMaxRowBlocks * ldb);
  counter.alloc(nt);
  out.alloc((size_t)2 * ldb);
  Scratch sc{partial.p, counter.p};
  pl->invb.assign(sp->nlev(), std::vector<double>(nn, 0.0));
  pl->mshare.assign(sp->nlev(), std::vector<double>(nn, 0.0));
  pl->ia_mass = 1.0 / mass_interval_ratio(sp->p);
  for (int li = 1; li < sp->nlev(); ++li) {
    const Level &L = *sp->lev[li];
    const size_t n = (size_t)L.R * ldb;
    v.alloc(n);
    w.alloc(n);
    v2.alloc(n);
    hash_fill(L, v.p, ldb, nt, s);
    for (int itp = 0; itp < kPowerIters; ++itp) {
      apply_level<double>(L, GF_APPLY_STENCIL, v.p, w.p, dsig.p, one.p, ldb, nt, nullptr, s, false);
      div_diag(L, v2.p, w.p, dsig.p, ldb, nt, s);
      if (itp + 1 < kPowerIters) std::swap(v.p, v2.p);
    }
    // lambda ~ (w . v_{k+1}) / (w . v_k) with w = A v_k, v_{k+1} = D^-1 w
    reduce_dot2<double, double, double>(L, v.p, w.p, v2.p, sc, ldb, nt, nullptr, nullptr, OP_STORE, 0.0, 0,
                                        out.p, s);
    std::vector<double> ho(2 * ldb);
    HIPCHK(hipMemcpyAsync(ho.data(), out.p, 2 * ldb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k < nn; ++k) {
      const double lam = ho[ldb + k] / ho[k];
      if (!(lam > 0.0) || !std::isfinite(lam)) fail(GF_EDEVICE, "spectral bound estimate failed");
      pl->invb[li][k] = 1.0 / (kChebSafety * lam);
      pl->mshare[li][k] = sig[k] * L.dM_mean / (sig[k] * L.dM_mean + L.dS_mean);
    }
    v.release();
    w.release();
    v2.release();
  }
  // coarse factors
  DBuf<double> sn;
  sn.upload(sig, s);
  DBuf<double> Lf;
  Lf.alloc((size_t)nn * sp->N0 * sp->N0);
  DBuf<int> info;
  info.alloc(nn);
  launch_coarse_factor(sp->M0.p, sp->S0.p, sp->N0, sn.p, nn, Lf.p, info.p, s);
  std::vector<int> hinfo(nn);
  HIPCHK(hipMemcpyAsync(hinfo.data(), info.p, nn * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < nn; ++k)
    if (hinfo[k] != 0) fail(GF_EINVAL, "coarse matrix not positive definite (shift too small)");
  // the solve applies the inverse (a dense matrix-vector product per system, all rows in parallel)
  pl->Ainv.alloc((size_t)nn * sp->N0 * sp->N0);
  launch_coarse_inverse(Lf.p, sp->N0, nn, pl->Ainv.p, s);
  HIPCHK(hipStreamSynchronize(s));
  pl->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  pl->last = sp->calls;
  Plan &ref = *pl;
  sp->plans[key] = std::move(pl);
  return ref;
}

// ------------------------------------------------------------------ batched MG-PCG
struct SolveSpec {
  int ncols = 0;                 // real systems (columns 0..ncols-1)
  std::vector<double> col_sig;   // shift per column
  std::vector<int> col_node;     // plan node per column
  const Plan *plan = nullptr;
  int prec = GF_PREC_FP64;
  int kind = GF_APPLY_STENCIL;
  int cheb = 2;
  double rtol = 1e-10;
  int max_iter = 500;
  int flags = 0;
  // operator M + sigma I (I the identity of the global unknowns) with a Jacobi preconditioner,
  // FP64, no multigrid plan (the shifted mass systems of the square root of M)
  bool mass_shift = false;
  int precond = GF_PRECOND_VCYCLE;
  bool cheb_auto = false;  // the caller left the degree to the library (set by prepare from the size)
  // the load has already passed through the inverse operator (an order of at least 1.5 in powers of
  // A^-1): it has little high-frequency content, and the smoothing interval stays [b/8, b] on every
  // node
  bool smooth_load = false;
  // the load is dL/du of a loss over point values (the first adjoint solve): rough, with much
  // high-frequency content; the automatic degree is the higher one of small batches
  bool rough_load = false;
};

struct SolveResult {
  int max_it = 0;
  double max_rel = 0.0;
  int flags = 0;
  double apply_ms = 0.0;
  int apply_launches = 0;
  double apply_col_sum = 0.0;
  double apply_bytes = 0.0;
  double smooth_ms = 0.0;
  int smooth_launches = 0;
  double smooth_bytes = 0.0;
};

// Chebyshev recurrence coefficients for interval [b ia, b], in units of 1/b
// alpha of the stiffness-dominated nodes by the degree of the smoothing polynomial: a polynomial of
// degree five or more damps a wider part of the spectrum, and [b/32, b] gave the fewest seconds per
// sample (degree 3, 64^2 elements per patch, 656 systems: 276 samples/s against 259 with alpha = 8
// and 283 / 267 with 48 / 64; the perturbed-sphere batch of 18 requests: 706 against 656; the
// torus: 1076 against 885); for degrees up to four alpha = 8 stays (degree 2, 64^2, 2,624 systems
// at degree four: 968 against 834 with 32; at degree three alpha = 16 gave 924 against 1023)
constexpr double kChebAlphaWide = 32.0;
constexpr int kChebWideFrom = 5;
static double alpha_for_degree(int deg) { return deg >= kChebWideFrom ? kChebAlphaWide : kChebAlpha; }

// lower end / upper end of the smoothing interval of node k on level li for a polynomial of degree deg
static double interval_ia(const Plan &pl, int li, int k, int deg) {
  const double rm = pl.mshare[li][k];
  return (1.0 - rm) / alpha_for_degree(deg) + rm * pl.ia_mass;
}

static void cheb_coeffs(int deg, double ia, std::vector<double> &c1, std::vector<double> &c2) {
  const double theta = (1.0 + ia) / 2.0, delta = (1.0 - ia) / 2.0, sigma1 = theta / delta;
  c1.assign(deg, 0.0);
  c2.assign(deg, 0.0);
  double rho_prev = 1.0 / sigma1;
  c2[0] = 1.0 / theta;
  for (int k = 1; k < deg; ++k) {
    const double rho = 1.0 / (2.0 * sigma1 - rho_prev);
    c1[k] = rho * rho_prev;
    c2[k] = 2.0 * rho / delta;
    rho_prev = rho;
  }
}

// smoothing degree of level li: spec.cheb on the finest level; below it, where each smoothing step is
// cheap in bytes but a full round of launches, one step (two on levels with more than kChebTwoRows
// patch rows).  Measured on the workloads of bench.py: the CG iteration count is set by the finest
// level's smoothing, and fewer coarse steps save time (degree 2, 64^2 elements per patch: 1017
// samples/s against 962 with two steps on every level).  A smooth load (SolveSpec::smooth_load) leaves
// an error made mostly of low frequencies, which the coarse levels carry: two steps on every level
// there (degree 3, 256^2 elements, beta = 2.3: 71.6 samples/s against 65.2).
static int level_degree(const gf_space *sp, const SolveSpec &spec, int li) {
  const Level &L = *sp->lev[li];
  if (li + 1 < sp->nlev())
    return std::min(spec.cheb, ((double)L.npatch * L.n1 * L.n1 > kChebTwoRows || spec.smooth_load) ? 2 : 1);
  return spec.cheb;
}

// Multigrid V-cycle on level li for the assembled right-hand side rsrc (type TR; converted to T into
// rconv when the types differ).  Pre-smoothing: Chebyshev-Jacobi from zero; coarse correction with
// the knot-insertion restriction of the residual, recursion, prolongation; post-smoothing with the
// same polynomial (a symmetric preconditioner).  Returns the buffer holding the result.  With
// fin_op >= 0 the last smoothing step also reduces r . z (and z . fin_q when fin_q is given) and
// applies fin_op (then *fused = true).
template <typename T, typename TR>
static T *vcycle(gf_space *sp, Workspace &w, const SolveSpec &spec, int li, const TR *rsrc, T *rconv, int fin_op,
                 bool *fused, hipStream_t s, const double *fin_q = nullptr) {
  const Level &L = *sp->lev[li];
  const int ldb = w.ldb, nt = w.ntiles;
  int *act = w.active.p;
  LevelWork &lw = w.lw[li];
  T *za = Prec<T>::za(lw), *zb = Prec<T>::zb(lw);
  if (fused) *fused = false;
  if (li == 0) {
    const T *r = (const T *)rsrc;
    if (rconv) {
      convert_rows<TR, T>(L, rsrc, rconv, ldb, nt, act, s);
      r = rconv;
    }
    coarse_solve<T>(L, sp->N0, za, r, spec.plan->Ainv.p, w.node.p, ldb, nt, act, s);
    return za;
  }
  const T *r = rconv ? (const T *)rconv : (const T *)rsrc;
  T *a = Prec<T>::a(lw);
  const T *cf = Prec<T>::cf(lw);
  const T *dM = Prec<T>::dM(L), *dS = Prec<T>::dS(L), *sig = Prec<T>::sig(w), *one = Prec<T>::one(w);
  Scratch sc = w.scratch();
  const int deg = level_degree(sp, spec, li);
  // Three-term recurrence: a step with a previous direction takes it as z - z_prev, z_prev being the
  // iterate before its input, which the output buffer still holds (the two iterate buffers swap
  // after every step); the first step after the start from zero takes it from the iterate itself
  // (dflags bit 0)
  auto smooth = [&](int k, bool last, int dflags) {
    EpiArgs<T> e;
    e.kind = EPI_CHEB;
    e.nslot = w.nslot;
    e.rows16 = w.rows16;
    e.dflags = dflags | (k > 0 ? 4 : 0);
    e.y = a;
    e.zout = zb;
    e.r = r;
    e.dM = dM;
    e.dS = dS;
    e.sig = sig;
    e.cf1 = cf + (size_t)k * ldb;
    e.cf2 = cf + (size_t)(deg + k) * ldb;
    if (last && fin_op >= 0) {
      e.dot = fin_q ? 2 : 1;
      e.q2 = fin_q;
      e.op = fin_op;
      if (fused) *fused = true;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (w.slog && li + 1 == sp->nlev()) {
      HIPCHK(hipEventCreate(&ev0));
      HIPCHK(hipEventCreate(&ev1));
      // read z, r (and z_prev), write z_out; with the two inner products also the FP64 vector q
      const int vecs = 3 + ((k > 0 && !(dflags & 1)) ? 1 : 0) + (e.dot == 2 ? (int)(sizeof(double) / sizeof(T)) : 0);
      w.slog->entries.push_back({ev0, ev1, vecs, (int)sizeof(T), w.slog->first_phase});
    }
    apply_epi<T>(L, spec.kind, za, sig, one, e, sc, w.cs.p, act, ldb, nt, spec.rtol * spec.rtol, spec.max_iter, s,
                 ev0, ev1);
    std::swap(za, zb);
  };
  // pre-smoothing from zero (the second step's previous direction is the first iterate itself); in
  // an outer-CG iteration the finest level's first step also updates the residual and tests it
  bool fused_first = false;
  if constexpr (std::is_same<TR, double>::value) {
    if (w.fuse_q && li + 1 == sp->nlev()) {
      cheb_first_cg<T>(L, w.r.p, w.fuse_q, rconv, za, dM, dS, sig, cf + (size_t)deg * ldb, sc, w.cs.p, act,
                       w.active0.p, ldb, nt, spec.rtol * spec.rtol, spec.max_iter, s);
      fused_first = true;
    }
  }
  if (!fused_first) {
    const bool bb = w.fuse_bb && li + 1 == sp->nlev() && std::is_same<TR, double>::value;
    cheb_first<T, TR>(L, rsrc, rconv, za, dM, dS, sig, cf + (size_t)deg * ldb, ldb, nt, act, s, bb ? &sc : nullptr,
                      bb ? w.cs.p : nullptr);
  }
  for (int k = 1; k < deg; ++k) smooth(k, false, k == 1 ? 1 : 0);
  // residual, restriction, coarse correction, prolongation
  {
    EpiArgs<T> e;
    e.kind = EPI_RESID;
    e.nslot = w.nslot;
    e.rows16 = w.rows16;
    e.y = a;
    e.r = r;
    apply_epi<T>(L, spec.kind, za, sig, one, e, sc, w.cs.p, act, ldb, nt, 0.0, 0, s);
  }
  const Level &C = *sp->lev[li - 1];
  T *rc = Prec<T>::r(w.lw[li - 1]);
  restrict_residual<T>(L, C, rc, a, nullptr, ldb, nt, act, s);
  launch_interface_sum<T>(C, rc, ldb, nt, act, s);
  T *zc = vcycle<T, T>(sp, w, spec, li - 1, rc, nullptr, -1, nullptr, s);
  prolong_add<T>(L, C, za, zc, ldb, nt, act, s);
  // post-smoothing
  for (int k = 0; k < deg; ++k) smooth(k, k == deg - 1, 0);
  return za;
}

// Additive multilevel (BPX) preconditioner: z = sum over the levels l of P_l D_l^-1 P_l^T r with
// D_l the diagonal of sigma M_l + S_l, and the exact (dense) solve on level 0.  The residual is
// restricted level by level (knot-insertion transposes, interface sums); on the way up every level
// adds its diagonally scaled residual to the prolongation of the coarser correction.
template <typename T, typename TR>
static T *bpx(gf_space *sp, Workspace &w, const SolveSpec &spec, const TR *rsrc, T *rconv, hipStream_t s) {
  const int fi = sp->nlev() - 1;
  const int ldb = w.ldb, nt = w.ntiles;
  int *act = w.active.p;
  const T *rf = (const T *)rsrc;
  if (rconv) {
    convert_rows<TR, T>(*sp->lev[fi], rsrc, rconv, ldb, nt, act, s);
    rf = rconv;
  }
  auto resid = [&](int l) -> const T * { return l == fi ? rf : Prec<T>::r(w.lw[l]); };
  for (int l = fi; l >= 1; --l) {
    const Level &L = *sp->lev[l], &C = *sp->lev[l - 1];
    T *rc = Prec<T>::r(w.lw[l - 1]);
    restrict_residual<T>(L, C, rc, resid(l), nullptr, ldb, nt, act, s);
    launch_interface_sum<T>(C, rc, ldb, nt, act, s);
  }
  T *zc = Prec<T>::za(w.lw[0]);
  coarse_solve<T>(*sp->lev[0], sp->N0, zc, Prec<T>::r(w.lw[0]), spec.plan->Ainv.p, w.node.p, ldb, nt, act, s);
  for (int l = 1; l <= fi; ++l) {
    const Level &L = *sp->lev[l], &C = *sp->lev[l - 1];
    T *z = Prec<T>::za(w.lw[l]);
    diag_scale<T>(L, z, resid(l), Prec<T>::sig(w), Prec<T>::dM(L), Prec<T>::dS(L), ldb, nt, act, s);
    prolong_add<T>(L, C, z, zc, ldb, nt, act, s);
    zc = z;
  }
  return zc;
}

// One batch of shifted systems (sigma_c M + S) x_c = r_c, one per column, on one space: on entry
// w.r holds the right-hand sides (assembled, patch-local layout), on exit w.x the solutions.
// prepare() and start() run eagerly; iterate() enqueues one CG iteration and is what the graph
// captures.
struct BatchSolve {
  gf_space *sp = nullptr;
  Workspace *w = nullptr;
  SolveSpec spec;
  SolveResult res;
  double *zd = nullptr;
  float *zf = nullptr;
  std::vector<hipEvent_t> evs;  // timed outer applies (pairs)
  SmoothLog slog;               // timed finest-level smoothing launches
  bool done = false;

  bool mixed() const { return spec.prec == GF_PREC_MIXED; }
  double tol2() const { return spec.rtol * spec.rtol; }
  // Mixed precision with the V-cycle on the stencil path: the search direction p is stored in FP32.
  // q = A p is still formed in FP64 from the stored p, and x += alpha p, r -= alpha q use that same
  // p, so x and r stay consistent in FP64 (the attainable accuracy is unchanged); the rounding of
  // p = z + beta p only perturbs the direction, as the FP32 preconditioner already does, which the
  // flexible beta absorbs.  It halves the bytes of the operator's window vector and of p in the
  // x/p update.  Decided in start() from the batch (shift groups, offsets).
  bool p32 = false;

  int concurrent = 1;  // batches solved together in one call (their graph branches share the GPU)
  void prepare(hipStream_t s) {
    const Level &F = sp->fine();
    const int ldb = w->ldb;
    if (spec.cheb_auto)
      spec.cheb = concurrent > 1 ? kDefaultChebConcurrent
                  : ((double)spec.ncols * F.N < kSmallBatchWork || spec.rough_load) ? kDefaultChebSmall
                                                                                     : kDefaultCheb;
    std::vector<double> sig(ldb, 1.0);
    std::vector<float> sigf(ldb, 1.0f);
    std::vector<int> node(ldb, 0);
    std::vector<ColState> cs(ldb);
    for (int c = 0; c < ldb; ++c) {
      cs[c] = ColState{};
      cs[c].done = (c < spec.ncols) ? 0 : 1;
      if (c < spec.ncols) {
        sig[c] = spec.col_sig[c];
        node[c] = spec.col_node[c];
      }
      sigf[c] = (float)sig[c];
    }
    std::fill(w->active_h.begin(), w->active_h.end(), 0);
    for (int c = 0; c < spec.ncols; ++c) w->active_h[c / CT] = 1;
    // shift structure of the column tiles (padding columns carry the shift 1)
    w->nslot = 0;
    w->rows16 = 1;
    for (int t = 0; t < w->ntiles; ++t) {
      std::vector<double> d;
      for (int c = t * CT; c < (t + 1) * CT; ++c) {
        if (std::find(d.begin(), d.end(), sig[c]) == d.end()) d.push_back(sig[c]);
        if (c % 16 != 0 && sig[c] != sig[c - 1]) w->rows16 = 0;
      }
      w->nslot = std::max(w->nslot, (int)d.size());
    }
    w->sig64.upload(sig, s);
    w->sig32.upload(sigf, s);
    w->node.upload(node, s);
    w->cs.upload(cs, s);
    w->active.upload(w->active_h, s);
    // Chebyshev coefficients of every smoothing step per system (the interval depends on the node)
    for (int li = 1; li < sp->nlev() && !spec.mass_shift; ++li) {
      const int deg = level_degree(sp, spec, li);
      std::vector<double> cf((size_t)2 * deg * ldb, 0.0), c1, c2;
      for (int c = 0; c < spec.ncols; ++c) {
        const int k = node[c];
        cheb_coeffs(deg, spec.smooth_load ? 1.0 / kChebAlpha : interval_ia(*spec.plan, li, k, deg), c1, c2);
        for (int st = 0; st < deg; ++st) {
          cf[(size_t)st * ldb + c] = c1[st];
          cf[(size_t)(deg + st) * ldb + c] = c2[st] * spec.plan->invb[li][k];
        }
      }
      std::vector<float> cff(cf.begin(), cf.end());
      w->lw[li].cf64.upload(cf, s);
      w->lw[li].cf32.upload(cff, s);
    }
    HIPCHK(hipMemsetAsync(w->x.p, 0, (size_t)F.R * ldb * sizeof(double), s));
  }

  // z = B r.  The V-cycle fuses the reduction of fin_op into its last smoothing step: r.z (OP_RZ0,
  // OP_BETA; in mixed precision with r as its FP32 copy), r.z and z.q in mixed precision
  // (OP_BETA_FLEX).  Returns whether it did.
  bool precondition(int fin_op, hipStream_t s) {
    const int fi = sp->nlev() - 1;
    bool fused = false;
    if (spec.mass_shift) {  // z = D^-1 r, D = diag(M) + sigma diag(I)
      const Level &F = sp->fine();
      zd = w->lw[fi].z64a.p;
      div_diag2(F, zd, w->r.p, w->one64.p, F.dM.p, w->sig64.p, F.dI.p, w->ldb, w->ntiles, w->active.p, s);
      return false;
    }
    if (spec.precond == GF_PRECOND_BPX) {
      if (!mixed())
        zd = bpx<double, double>(sp, *w, spec, w->r.p, nullptr, s);
      else
        zf = bpx<float, double>(sp, *w, spec, w->r.p, w->lw[fi].r32.p, s);
      return false;
    }
    if (!mixed()) {
      zd = vcycle<double, double>(sp, *w, spec, fi, w->r.p, nullptr, fin_op, &fused, s);
    } else if (fin_op == OP_BETA_FLEX && fuse_flex()) {
      // the flexible beta's r.z and z.q from the last FP32 smoothing step (r as its FP32 copy)
      zf = vcycle<float, double>(sp, *w, spec, fi, w->r.p, w->lw[fi].r32.p, OP_BETA_FLEX, &fused, s, w->q.p);
    } else if (fin_op == OP_RZ0 && fuse_flex()) {
      // the first r.z the same way (the flexible beta divides by it)
      zf = vcycle<float, double>(sp, *w, spec, fi, w->r.p, w->lw[fi].r32.p, OP_RZ0, &fused, s);
    } else {
      zf = vcycle<float, double>(sp, *w, spec, fi, w->r.p, w->lw[fi].r32.p, -1, nullptr, s);
    }
    return fused;
  }

  // whether the mixed-precision V-cycle can take the flexible beta's two inner products in its last
  // smoothing step (stencil path on at least two levels, offsets within the kernel's 32-bit range)
  bool fuse_flex() const {
    return spec.kind == GF_APPLY_STENCIL && sp->nlev() > 1 && stencil_dot2_fits(sp->fine(), w->ldb);
  }

  void start(hipStream_t s) {
    const Level &F = sp->fine();
    p32 = mixed() && !spec.mass_shift && spec.kind == GF_APPLY_STENCIL && spec.precond == GF_PRECOND_VCYCLE &&
          sp->nlev() > 1 && w->rows16 && w->p32.p && outer_p32_fits(F, w->ldb);
    // the smoothing launches of the first preconditioner application are timed with the others
    w->slog = (spec.flags & GF_FLAG_TIME_APPLY) ? &slog : nullptr;
    slog.first_phase = true;
    const int ldb = w->ldb, nt = w->ntiles;
    Scratch sc = w->scratch();
    // |b|^2: taken by the V-cycle's first finest-level step where there is one, else a reduction pass
    w->fuse_bb = spec.precond == GF_PRECOND_VCYCLE && !spec.mass_shift && sp->nlev() > 1;
    if (!w->fuse_bb)
      reduce_dot<double, double>(F, w->r.p, w->r.p, sc, ldb, nt, w->cs.p, w->active.p, OP_BB, tol2(),
                                 spec.max_iter, nullptr, s);
    const bool fused_rz0 = precondition(OP_RZ0, s);
    w->fuse_bb = false;
    if (!fused_rz0) {
      if (mixed())
        reduce_dot<double, float>(F, w->r.p, zf, sc, ldb, nt, w->cs.p, w->active.p, OP_RZ0, tol2(), spec.max_iter,
                                  nullptr, s);
      else
        reduce_dot<double, double>(F, w->r.p, zd, sc, ldb, nt, w->cs.p, w->active.p, OP_RZ0, tol2(),
                                   spec.max_iter, nullptr, s);
    }
    if (p32)
      convert_rows<float, float>(F, zf, w->p32.p, ldb, nt, w->active.p, s);
    else if (mixed())
      convert_rows<float, double>(F, zf, w->p.p, ldb, nt, w->active.p, s);
    else
      convert_rows<double, double>(F, zd, w->p.p, ldb, nt, w->active.p, s);
  }

  // one CG iteration: q = A p (+ p.q -> alpha), x += alpha p, r -= alpha q (+ |r|^2 -> test),
  // z = B r (+ r.z -> beta), p = z + beta p.  With the V-cycle the residual update and the test run
  // inside its first kernel and x += alpha p with the update of p (two passes over the batch fewer).
  void iterate(hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const Level &F = sp->fine();
    const int ldb = w->ldb, nt = w->ntiles;
    Scratch sc = w->scratch();
    EpiArgs<double> e;
    e.kind = EPI_STORE;
    e.nslot = w->nslot;
    e.rows16 = w->rows16;
    e.y = w->q.p;
    e.dot = 1;
    e.op = OP_ALPHA;
    if (spec.mass_shift) {
      apply_epi<double>(F, GF_APPLY_STENCIL, w->p.p, w->one64.p, w->sig64.p, e, sc, w->cs.p, w->active.p, ldb, nt,
                        tol2(), spec.max_iter, s, e0, e1, F.stI.p);
    } else if (p32) {
      const ApplyTune &t = get_tune_p32(F, ldb, nt, w->sig64.p, w->one64.p, e, s);
      apply_outer_p32(F, w->p32.p, w->sig64.p, w->one64.p, e, sc, w->cs.p, w->active.p, ldb, nt, tol2(),
                      spec.max_iter, s, t, e0, e1);
    } else {
      apply_epi<double>(F, spec.kind, w->p.p, w->sig64.p, w->one64.p, e, sc, w->cs.p, w->active.p, ldb, nt, tol2(),
                        spec.max_iter, s, e0, e1);
    }
    if (spec.mass_shift) {
      // Jacobi CG of M + sigma I: residual update, z = r / D, the test and beta in one pass
      zd = w->lw[sp->nlev() - 1].z64a.p;
      jacobi_step(F, w->r.p, w->q.p, zd, w->one64.p, F.dM.p, w->sig64.p, F.dI.p, sc, w->cs.p, w->active.p,
                  w->active0.p, ldb, nt, tol2(), spec.max_iter, s);
      update_xp<double>(F, w->x.p, w->p.p, zd, w->cs.p, w->active0.p, ldb, nt, s);
      return;
    }
    // (a one-level space has no smoothing step to carry the update: the coarse solve is the V-cycle)
    const bool fuse = !spec.mass_shift && spec.precond == GF_PRECOND_VCYCLE && sp->nlev() > 1;
    if (fuse)
      w->fuse_q = w->q.p;
    else
      update_xr2(F, w->x.p, w->r.p, w->p.p, w->q.p, sc, ldb, nt, w->cs.p, w->active.p, tol2(), spec.max_iter, s);
    if (mixed()) {
      const bool fused_dot = precondition(OP_BETA_FLEX, s);
      w->fuse_q = nullptr;
      if (!fused_dot)
        reduce_dot2<double, float, double>(F, w->r.p, zf, w->q.p, sc, ldb, nt, w->cs.p, w->active.p, OP_BETA_FLEX,
                                           tol2(), spec.max_iter, nullptr, s);
      if (p32)
        update_xp<float, float>(F, w->x.p, w->p32.p, zf, w->cs.p, w->active0.p, ldb, nt, s);
      else if (fuse)
        update_xp<float>(F, w->x.p, w->p.p, zf, w->cs.p, w->active0.p, ldb, nt, s);
      else
        update_p2<float>(F, w->p.p, zf, w->cs.p, ldb, nt, w->active.p, s);
    } else {
      const bool fused_dot = precondition(OP_BETA, s);
      w->fuse_q = nullptr;
      if (!fused_dot)
        reduce_dot<double, double>(F, w->r.p, zd, sc, ldb, nt, w->cs.p, w->active.p, OP_BETA, tol2(),
                                   spec.max_iter, nullptr, s);
      if (fuse)
        update_xp<double>(F, w->x.p, w->p.p, zd, w->cs.p, w->active0.p, ldb, nt, s);
      else
        update_p2<double>(F, w->p.p, zd, w->cs.p, ldb, nt, w->active.p, s);
    }
  }

  void new_event_pair(hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    w->slog = (spec.flags & GF_FLAG_TIME_APPLY) ? &slog : nullptr;
    slog.first_phase = false;
    if (!(spec.flags & GF_FLAG_TIME_APPLY)) return;
    HIPCHK(hipEventCreate(e0));
    HIPCHK(hipEventCreate(e1));
    evs.push_back(*e0);
    evs.push_back(*e1);
  }

  // read the timed pairs recorded since the last call (the stream is synchronised)
  // prev_tiles: column tiles active when the iteration began (the outer operator's launches and the
  // first preconditioner application); now_tiles: active after its convergence test (the V-cycle
  // that follows the test skips the tiles that converged)
  void harvest_events(int prev_tiles, int now_tiles) {
    const int active_tiles = prev_tiles;
    for (size_t i = 0; i + 1 < evs.size(); i += 2) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      res.apply_ms += ms;
      res.apply_launches += 1;
      res.apply_col_sum += (double)active_tiles * CT;
      // algorithmic bytes: read x (FP32 when the search direction is stored so) and write y (FP64)
      // for every active column of every patch row, plus the two FP64 stencils of every row
      const Level &F = sp->fine();
      const double rows = (double)F.npatch * F.n1 * F.n1;
      res.apply_bytes += ((p32 ? 4.0 : 8.0) + 8.0) * active_tiles * CT * rows + 2.0 * F.S * F.S * 8.0 * rows;
    }
    const Level &F = sp->fine();
    const double rows = (double)F.npatch * F.n1 * F.n1;
    for (auto &e : slog.entries) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e.e0, e.e1));
      res.smooth_ms += ms;
      res.smooth_launches += 1;
      // algorithmic bytes: the batch vectors read and written per active column and patch row, plus
      // the two stencils per row
      const int tiles = e.first ? prev_tiles : now_tiles;
      res.smooth_bytes += (double)e.vecs * e.elem * tiles * CT * rows + 2.0 * F.S * F.S * e.elem * rows;
    }
    slog.clear();
  }

  int active_tiles() const {
    int a = 0;
    for (int t = 0; t < w->ntiles; ++t) a += w->active_h[t] ? 1 : 0;
    return a;
  }

  void read_active(hipStream_t s) {
    HIPCHK(hipMemcpyAsync(w->active_h.data(), w->active.p, w->ntiles * sizeof(int), hipMemcpyDeviceToHost, s));
  }

  void collect() {
    for (auto e : evs) (void)hipEventDestroy(e);
    evs.clear();
    slog.clear();
    w->slog = nullptr;
    const int ldb = w->ldb;
    std::vector<ColState> out(ldb);
    HIPCHK(hipMemcpy(out.data(), w->cs.p, ldb * sizeof(ColState), hipMemcpyDeviceToHost));
    for (int c = 0; c < spec.ncols; ++c) {
      res.max_it = std::max(res.max_it, out[c].it);
      const double rel = out[c].bb > 0 ? std::sqrt(out[c].rr / out[c].bb) : 0.0;
      res.max_rel = std::max(res.max_rel, rel);
      res.flags |= out[c].flag;
      if (!out[c].done) res.flags |= 1;
    }
  }
};

// side streams of a context for the parallel branches of a multi-problem graph (default priority)
static std::vector<hipStream_t> &side_streams(gf_context *ctx, size_t n) {
  static std::map<gf_context *, std::vector<hipStream_t>> m;
  auto &v = m[ctx];
  while (v.size() < n) {
    hipStream_t st;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    v.push_back(st);
  }
  return v;
}

// "some column tile still active" into one word: zeroed at the start of a chunk, set by any tile
__global__ void k_flag_zero(int *flag) { *flag = 0; }
__global__ void k_flag_any(const int *active, int n, int *flag) {
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    if (active[t]) *flag = 1;
}

constexpr int kGraphChunk = 4;    // CG iterations per captured graph
constexpr size_t kMaxGraphs = 32;  // instantiated graphs kept per context

// Identity of a captured chunk: everything its kernels take as arguments -- the batches' spaces,
// plans, workspaces and their buffers, and the solver settings baked into the launches.
static std::string graph_key(const std::vector<BatchSolve *> &items, int chunk) {
  std::ostringstream os;
  os.precision(17);
  os << chunk;
  for (const BatchSolve *it : items) {
    const Workspace &w = *it->w;
    const SolveSpec &sp = it->spec;
    os << "|" << (const void *)it->sp << "," << (const void *)sp.plan << "," << (const void *)&w << "," << w.ldb
       << "," << sp.prec << "," << sp.kind << "," << sp.cheb << "," << sp.rtol << "," << sp.max_iter << ","
       << sp.flags << "," << sp.precond << "," << sp.mass_shift << "," << sp.smooth_load << "," << w.nslot << ","
       << w.rows16 << "," << it->p32 << "," << (const void *)w.x.p << "," << (const void *)w.r.p << ","
       << (const void *)w.p.p << "," << (const void *)w.p32.p << "," << (const void *)w.q.p << "," << (const void *)w.cs.p << "," << (const void *)w.partial.p << ","
       << (const void *)w.active.p << "," << (const void *)w.sig64.p;
    if (sp.plan) os << "," << (const void *)sp.plan->Ainv.p;
    for (const LevelWork &l : w.lw)
      os << "," << (const void *)l.z64a.p << (const void *)l.z32a.p << (const void *)l.cf64.p << (const void *)l.cf32.p;
  }
  return os.str();
}

static void graph_destroy(gf_context::Graph &gr) {
  if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
  if (gr.graph) (void)hipGraphDestroy(gr.graph);
  for (hipEvent_t e : gr.events) (void)hipEventDestroy(e);
  gr.exec = nullptr;
  gr.graph = nullptr;
  gr.events.clear();
}

// drop the cached graphs that use space sp (its workspaces are about to be freed)
static void drop_graphs_of(gf_context *ctx, const gf_space *sp) {
  if (!ctx) return;
  for (auto it = ctx->graphs.begin(); it != ctx->graphs.end();) {
    if (std::find(it->second.spaces.begin(), it->second.spaces.end(), (const void *)sp) != it->second.spaces.end()) {
      graph_destroy(it->second);
      it = ctx->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// Bounds of a space's caches of plans (by the bytes of their coarse inverses) and workspaces (by the
// bytes of their batch vectors).  At the start of every call that uses the space, the least recently
// used entries are released until each cache fits its bound again (the ones the new call builds come
// on top until the next call).  Nothing cached is released during a call, and no pointer into the
// caches outlives a call: the cached graphs that use the space are dropped with them, and tapes own
// their saved solutions.  A loop over new values of kappa (a new chain plan and node plan on every
// call) thus keeps its device memory bounded, while repeated calls with the same batches keep theirs.
// The environment variables GF_PLAN_CACHE_MB and GF_WORKSPACE_CACHE_MB set other bounds (MiB).
constexpr size_t kPlanCacheBytes = (size_t)1 << 30;
constexpr size_t kWorkspaceCacheBytes = (size_t)96 << 30;

static size_t cache_bound(const char *env, size_t dflt) {
  const char *v = std::getenv(env);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  const double mb = std::strtod(v, &end);
  if (end == v || !(mb >= 0.0) || !std::isfinite(mb)) return dflt;
  return (size_t)(mb * 1048576.0);
}

static void begin_call(gf_space *sp) {
  ++sp->calls;
  const size_t plan_bound = cache_bound("GF_PLAN_CACHE_MB", kPlanCacheBytes);
  const size_t ws_bound = cache_bound("GF_WORKSPACE_CACHE_MB", kWorkspaceCacheBytes);
  size_t pb = 0, wb = 0;
  for (const auto &kv : sp->plans) pb += kv.second->Ainv.n * sizeof(double);
  auto reg = ws_registry().find(sp);
  if (reg != ws_registry().end() && reg->second)
    for (const auto &kv : reg->second->m) wb += kv.second->bytes;
  if (pb <= plan_bound && wb <= ws_bound) return;
  // the work of earlier calls that reads them is finished (their results were returned) but not
  // necessarily retired on the device
  HIPCHK(hipStreamSynchronize(sp->ctx->stream));
  drop_graphs_of(sp->ctx, sp);
  while (pb > plan_bound && !sp->plans.empty()) {
    auto lru = sp->plans.begin();
    for (auto it = sp->plans.begin(); it != sp->plans.end(); ++it)
      if (it->second->last < lru->second->last) lru = it;
    pb -= lru->second->Ainv.n * sizeof(double);
    sp->plans.erase(lru);
  }
  if (reg != ws_registry().end() && reg->second) {
    auto &m = reg->second->m;
    while (wb > ws_bound && !m.empty()) {
      auto lru = m.begin();
      for (auto it = m.begin(); it != m.end(); ++it)
        if (it->second->last < lru->second->last) lru = it;
      wb -= lru->second->bytes;
      m.erase(lru);
    }
  }
}

// Runs the CG iterations of all batches together.  The first iteration is enqueued eagerly (it also
// runs the launch-shape autotuner).  Then kGraphChunk iterations of every batch are captured into one
// HIP graph -- one branch per batch, forked from and joined back into the capture stream, each branch
// running its batch's iterations in sequence -- followed by the reduction of every batch's active-tile
// flags into one word.  The graph is replayed until no tile is active: one read-back of that word and
// one host synchronisation per chunk.  Converged column tiles exit at the top of every kernel, so the
// iterations of a chunk after convergence cost only their launches.  Instantiated graphs are kept in
// the context, keyed by everything their launches take as arguments, and reused by later calls.
// Smoothing degree of a batch solved alone with at least kTuneMinWork columns x unknowns (the caller
// leaving the degree to the library): on its first solve the batch is solved once with every
// candidate degree, eagerly from its own right-hand side, and timed with HIP events to convergence;
// the fastest degree is kept for the space and the batch configuration (shifts, width, precision,
// tolerance, load), so later calls with the same batch reuse it.  The right-hand side is restored
// before the solve proper.  (Predicting the iteration count from the residual reduction of the first
// few iterations favoured high degrees that were slower to convergence.)  A batch below
// kSmallBatchWork (one column tile on a large mesh, such as a step of the integer chain) is bound by
// latency rather than memory traffic, and its candidates reach the high degrees that cut the
// iterations.  Smaller batches, whose solves take a few milliseconds, and concurrent batches, which
// share the GPU, keep the fixed degrees of prepare().
constexpr int kTuneDegrees[] = {2, 3, 4, 5};
constexpr int kTuneDegreesSmall[] = {3, 5, 7, 9};
constexpr double kTuneMinWork = 1e7;

static void tune_degree(hipStream_t s, BatchSolve &b) {
  const SolveSpec &sp0 = b.spec;
  const Level &F = b.sp->fine();
  if (!sp0.cheb_auto || sp0.mass_shift || sp0.precond != GF_PRECOND_VCYCLE || b.sp->nlev() < 2 ||
      b.concurrent > 1 || sp0.kind != GF_APPLY_STENCIL || !sp0.plan ||
      (double)sp0.ncols * F.N < kTuneMinWork)
    return;
  const bool small = (double)sp0.ncols * F.N < kSmallBatchWork;
  std::ostringstream key;
  key.precision(17);
  key << b.w->ldb << "," << sp0.ncols << "," << sp0.prec << "," << sp0.rtol << "," << sp0.max_iter << ","
      << sp0.rough_load << "," << sp0.smooth_load << "," << plan_key(sp0.plan->sig) << "|";
  for (int c = 0; c < sp0.ncols; ++c) key << sp0.col_node[c] << ",";
  auto it = b.sp->cheb_tuned.find(key.str());
  if (it == b.sp->cheb_tuned.end()) {
    const size_t nr = (size_t)F.R * b.w->ldb;
    DBuf<double> r0;
    r0.alloc(nr);
    HIPCHK(hipMemcpyAsync(r0.p, b.w->r.p, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    const int flags0 = b.spec.flags;
    b.spec.flags &= ~GF_FLAG_TIME_APPLY;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = kDefaultCheb;
    float best_ms = 1e30f;
    // untimed warm-up iteration: the launch-shape autotuner runs on the first use of each kernel
    b.spec.cheb = kDefaultCheb;
    b.spec.cheb_auto = false;
    b.prepare(s);
    b.start(s);
    b.iterate(s, nullptr, nullptr);
    const std::vector<int> cand = small ? std::vector<int>(std::begin(kTuneDegreesSmall), std::end(kTuneDegreesSmall))
                                        : std::vector<int>(std::begin(kTuneDegrees), std::end(kTuneDegrees));
    for (int deg : cand) {
      b.spec.cheb = deg;
      b.spec.cheb_auto = false;
      HIPCHK(hipMemcpyAsync(b.w->r.p, r0.p, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
      b.prepare(s);
      HIPCHK(hipEventRecord(e0, s));
      b.start(s);
      int its = 0;
      while (its < b.spec.max_iter) {
        b.iterate(s, nullptr, nullptr);
        ++its;
        b.read_active(s);
        HIPCHK(hipStreamSynchronize(s));
        if (b.active_tiles() == 0) break;
      }
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (std::getenv("GF_TUNE_LOG"))
        std::fprintf(stderr, "degree tune p=%d lev=%d cols=%d deg=%d: %d iterations, %.2f ms\n", b.sp->p, b.sp->j,
                     sp0.ncols, deg, its, ms);
      if (ms < best_ms) {
        best_ms = ms;
        best = deg;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipMemcpyAsync(b.w->r.p, r0.p, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    b.spec.flags = flags0;
    it = b.sp->cheb_tuned.emplace(key.str(), best).first;
  }
  b.spec.cheb = it->second;
  b.spec.cheb_auto = false;
}

static void solve_all(gf_context *ctx, std::vector<BatchSolve *> &items, bool use_graph) {
  hipStream_t s = ctx->stream;
  for (auto *it : items) it->concurrent = (int)items.size();
  for (auto *it : items) tune_degree(s, *it);
  for (auto *it : items) it->prepare(s);
  for (auto *it : items) it->start(s);
  int max_iter = 0;
  for (auto *it : items) max_iter = std::max(max_iter, it->spec.max_iter);
  auto all_done = [&]() {
    bool any = false;
    std::vector<int> prev(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
      prev[i] = items[i]->active_tiles();  // tiles the operator launches just processed
      items[i]->read_active(s);
    }
    HIPCHK(hipStreamSynchronize(s));
    ctx->host_syncs += 1;
    for (size_t i = 0; i < items.size(); ++i) items[i]->harvest_events(prev[i], items[i]->active_tiles());
    for (auto *it : items)
      for (int t = 0; t < it->w->ntiles; ++t) any = any || it->w->active_h[t];
    return !any;
  };
  // eager first iteration
  for (auto *it : items) {
    hipEvent_t e0, e1;
    it->new_event_pair(&e0, &e1);
    it->iterate(s, e0, e1);
  }
  if (all_done() || max_iter <= 1) {
    for (auto *it : items) it->collect();
    return;
  }
  for (auto *it : items) {
    for (auto e : it->evs) (void)hipEventDestroy(e);
    it->evs.clear();
  }
  if (!use_graph) {
    for (int k = 1; k < max_iter; ++k) {
      for (auto *it : items) {
        hipEvent_t e0, e1;
        it->new_event_pair(&e0, &e1);
        it->iterate(s, e0, e1);
      }
      const bool fin = all_done();
      for (auto *it : items) {
        for (auto e : it->evs) (void)hipEventDestroy(e);
        it->evs.clear();
      }
      if (fin) break;
    }
    for (auto *it : items) it->collect();
    return;
  }
  if (!ctx->flag_dev) {
    HIPCHK(hipMalloc((void **)&ctx->flag_dev, sizeof(int)));
    HIPCHK(hipHostMalloc((void **)&ctx->flag_host, sizeof(int), hipHostMallocDefault));
  }
  const std::string key = graph_key(items, kGraphChunk);
  auto found = ctx->graphs.find(key);
  if (found == ctx->graphs.end()) {
    for (auto *it : items) it->w->slog = nullptr;
    // capture on a side stream (the context stream may be the null stream, which cannot capture); the
    // graph is launched on the context stream, after all of its earlier work
    std::vector<hipStream_t> &side = side_streams(ctx, items.size() + 1);
    hipStream_t cap = side[0];
    std::vector<hipEvent_t> joins(items.size());
    hipEvent_t fork;
    HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (auto &j : joins) HIPCHK(hipEventCreateWithFlags(&j, hipEventDisableTiming));
    gf_context::Graph gr;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    try {
      hipLaunchKernelGGL(k_flag_zero, dim3(1), dim3(1), 0, cap, ctx->flag_dev);
      HIPCHK(hipEventRecord(fork, cap));
      for (size_t i = 0; i < items.size(); ++i) {
        HIPCHK(hipStreamWaitEvent(side[i + 1], fork, 0));
        for (int k = 0; k < kGraphChunk; ++k) items[i]->iterate(side[i + 1], nullptr, nullptr);
        HIPCHK(hipEventRecord(joins[i], side[i + 1]));
        HIPCHK(hipStreamWaitEvent(cap, joins[i], 0));
      }
      for (auto *it : items)
        hipLaunchKernelGGL(k_flag_any, dim3(1), dim3(256), 0, cap, it->w->active.p, it->w->ntiles, ctx->flag_dev);
      HIPCHK(hipGetLastError());
    } catch (...) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(cap, &g2);
      if (g2) (void)hipGraphDestroy(g2);
      (void)hipEventDestroy(fork);
      for (auto j : joins) (void)hipEventDestroy(j);
      throw;
    }
    HIPCHK(hipStreamEndCapture(cap, &gr.graph));
    // the events recorded during the capture live as long as the graph (released in graph_destroy)
    gr.events.push_back(fork);
    gr.events.insert(gr.events.end(), joins.begin(), joins.end());
    HIPCHK(hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0));
    for (auto *it : items)
      if (std::find(gr.spaces.begin(), gr.spaces.end(), (const void *)it->sp) == gr.spaces.end())
        gr.spaces.push_back(it->sp);
    if (ctx->graphs.size() >= kMaxGraphs) {  // drop the least recently used
      auto lru = ctx->graphs.begin();
      for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
        if (g->second.last < lru->second.last) lru = g;
      graph_destroy(lru->second);
      ctx->graphs.erase(lru);
    }
    found = ctx->graphs.emplace(key, gr).first;
  }
  found->second.last = ++ctx->graph_clock;
  for (int k = 1; k < max_iter; k += kGraphChunk) {
    HIPCHK(hipGraphLaunch(found->second.exec, s));
    HIPCHK(hipMemcpyAsync(ctx->flag_host, ctx->flag_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->host_syncs += 1;
    if (*ctx->flag_host == 0) break;
  }
  for (auto *it : items) it->collect();
}

static SolveResult solve_batch(gf_space *sp, Workspace &w, const SolveSpec &spec) {
  // per-launch HIP events need the eager path (events recorded inside a graph are not timed)
  const bool use_graph = !(spec.flags & (GF_FLAG_NO_GRAPH | GF_FLAG_TIME_APPLY));
  BatchSolve b;
  b.sp = sp;
  b.w = &w;
  b.spec = spec;
  std::vector<BatchSolve *> items{&b};
  solve_all(sp->ctx, items, use_graph);
  return b.res;
}

// ------------------------------------------------------------------ allocation-free operator apply
// Work space of gf_space_apply_noalloc: a file-scope device array (each GPU holds its own copy, at its
// own address, for the life of the process).  Host code never uses the array's name as a device
// address: the device address is looked up once per device (noalloc_register, from gf_context_create,
// with that device current) and passed to the kernels.  It holds the patch-local input and output
// batches [R][ldb] and the per-column coefficients; every call overwrites what it reads.
constexpr size_t kNoAllocBytes = (size_t)256 << 20;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (device index `device`), looked up once
static void noalloc_register(int device) {
  if (device < 0 || device >= kMaxDevices) fail(GF_EDEVICE, "device index above the supported range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  double *ptr = nullptr;
  HIPCHK(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(GF_EDEVICE, "no device address for the allocation-free work space");
  g_scratch_ptr[device] = ptr;
}

static double *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

__global__ void k_fill2(double *a, double va, double *b, double vb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a[i] = va;
    b[i] = vb;
  }
}

}  // namespace gf

using namespace gf;

// ================================================================== C ABI
extern "C" {

const char *gf_last_error(void) { return g_last_error.c_str(); }
int gf_abi_version(void) { return GF_ABI_VERSION; }

gf_status gf_probe_fma(gf_context *ctx, int32_t precision, double *tflops) {
  return guarded([&] {
    if (!ctx || !tflops) fail(GF_EINVAL, "null argument");
    if (precision != GF_PREC_FP64 && precision != GF_PREC_MIXED) fail(GF_EINVAL, "unknown precision");
    HIPCHK(hipSetDevice(ctx->device));
    *tflops = fma_probe(precision == GF_PREC_FP64, ctx->stream);
  });
}

gf_status gf_context_create(int32_t device, void *hip_stream, gf_context **out) {
  return guarded([&] {
    if (!out) fail(GF_EINVAL, "out is null");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) fail(GF_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) fail(GF_EDEVICE, "device index out of range");
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      fail(GF_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
    HIPCHK(hipSetDevice(device));
    noalloc_register(device);
    std::unique_ptr<gf_context> c(new gf_context());
    c->device = device;
    c->stream = (hipStream_t)hip_stream;  // NULL: the device's null stream
    *out = c.release();
  });
}

void gf_context_destroy(gf_context *ctx) {
  if (!ctx) return;
  for (auto &g : ctx->graphs) graph_destroy(g.second);
  ctx->graphs.clear();
  if (ctx->flag_dev) (void)hipFree(ctx->flag_dev);
  if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

gf_status gf_geometry_cubesphere(gf_context *ctx, double perturb_amp, gf_geometry **out) {
  return guarded([&] {
    if (!out) fail(GF_EINVAL, "null argument");
    *out = nullptr;
    if (!std::isfinite(perturb_amp) || !(std::fabs(perturb_amp) < 1.0))
      fail(GF_EINVAL, "perturb_amp must be finite with |perturb_amp| < 1");
    gf_geometry *g = new gf_geometry();
    g->ctx = ctx;
    g->amp = perturb_amp;
    *out = g;
  });
}

gf_status gf_geometry_nurbs(gf_context *ctx, int32_t npatch, int32_t deg_u, int32_t deg_v, const int32_t *ncoef,
                            const double *knots, const double *ctrl, gf_geometry **out) {
  return guarded([&] {
    if (!ncoef || !knots || !ctrl || !out) fail(GF_EINVAL, "null argument");
    *out = nullptr;
    if (npatch < 1 || npatch > 4096) fail(GF_EINVAL, "npatch must be in 1..4096");
    if (deg_u < 1 || deg_u > 4 || deg_v < 1 || deg_v > 4) fail(GF_EINVAL, "geometry degrees must be in 1..4");
    std::unique_ptr<gf_geometry> g(new gf_geometry());
    g->ctx = ctx;
    g->kind = SURF_NURBS;
    g->npatch = npatch;
    NurbsHost &h = g->nurbs;
    h.npatch = npatch;
    h.du = deg_u;
    h.dv = deg_v;
    int64_t koff = 0, coff = 0;
    // open knot vector on [0, 1]: deg+1 zeros, non-decreasing interior knots of multiplicity <= deg,
    // deg+1 ones
    auto check_knots = [&](const double *U, int n, int d) {
      for (int i = 0; i < n + d + 1; ++i)
        if (!std::isfinite(U[i])) fail(GF_EINVAL, "knot not finite");
      for (int i = 0; i <= d; ++i)
        if (U[i] != 0.0 || U[n + i] != 1.0) fail(GF_EINVAL, "knot vectors must be open on [0, 1]");
      for (int i = 0; i < n + d; ++i)
        if (U[i + 1] < U[i]) fail(GF_EINVAL, "knots must be non-decreasing");
      if (n > d + 1 && (U[d + 1] <= 0.0 || U[n - 1] >= 1.0)) fail(GF_EINVAL, "interior knots must lie in (0, 1)");
      for (int i = d + 1; i < n; ++i) {
        int mult = 1;
        while (i + mult < n && U[i + mult] == U[i]) ++mult;
        if (mult > d) fail(GF_EINVAL, "interior knot multiplicity exceeds the degree");
      }
    };
    for (int m = 0; m < npatch; ++m) {
      const int ns = ncoef[2 * m], nt = ncoef[2 * m + 1];
      if (ns < deg_u + 1 || nt < deg_v + 1 || ns > 4096 || nt > 4096)
        fail(GF_EINVAL, "control points per direction must be in degree+1..4096");
      const int64_t ku = koff, kv = koff + ns + deg_u + 1;
      check_knots(knots + ku, ns, deg_u);
      check_knots(knots + kv, nt, deg_v);
      for (int64_t i = 0; i < (int64_t)ns * nt; ++i) {
        const double *c = ctrl + 4 * (coff + i);
        for (int k = 0; k < 4; ++k)
          if (!std::isfinite(c[k])) fail(GF_EINVAL, "control point not finite");
        if (!(c[3] > 0.0)) fail(GF_EINVAL, "weights must be positive");
      }
      h.pinfo.insert(h.pinfo.end(), {ns, nt, (int)ku, (int)kv, (int)coff});
      koff = kv + nt + deg_v + 1;
      coff += (int64_t)ns * nt;
      if (koff > (int64_t)1 << 30 || coff > (int64_t)1 << 28) fail(GF_EINVAL, "geometry too large");
    }
    h.knots.assign(knots, knots + koff);
    h.ctrl.assign(ctrl, ctrl + 4 * coff);
    // the interfaces must be consistent before anything is built on them
    std::vector<int> l2g;
    int N = 0;
    glue_patches_nurbs(h, 1, 0, l2g, N);
    *out = g.release();
  });
}

int32_t gf_geometry_npatch(const gf_geometry *g) { return g ? g->npatch : -1; }

void gf_geometry_destroy(gf_geometry *g) {
  if (!g) return;
  if (--g->refs == 0) delete g;
}

gf_status gf_locate(const gf_geometry *geom, int32_t npts, const double *xyz, int32_t *patch, double *st) {
  return guarded([&] {
    if (!geom || (npts > 0 && (!xyz || !patch || !st)) || npts < 0) fail(GF_EINVAL, "bad arguments");
    if (geom->kind == SURF_NURBS) {
      for (int i = 0; i < npts; ++i) {
        const double P[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        if (!std::isfinite(P[0]) || !std::isfinite(P[1]) || !std::isfinite(P[2])) fail(GF_EINVAL, "point not finite");
        double s = 0, t = 0, dist = 0;
        int m = -1;
        nurbs_locate(geom->nurbs, P, &m, &s, &t, &dist);
        if (m < 0) fail(GF_EINVAL, "closest point not found (the surface evaluates to non-finite values)");
        patch[i] = m;
        st[2 * i] = s;
        st[2 * i + 1] = t;
      }
      return;
    }
    for (int i = 0; i < npts; ++i) {
      const double X[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
      int ax = 0;
      for (int k = 1; k < 3; ++k)
        if (std::fabs(X[k]) > std::fabs(X[ax])) ax = k;
      const double den = std::fabs(X[ax]);
      if (!(den > 0.0) || !std::isfinite(den)) fail(GF_EINVAL, "point at the origin or not finite");
      const int sign = X[ax] > 0 ? 1 : -1;
      int m = -1;
      for (int k = 0; k < 6; ++k)
        if (kPatchFrames[k].fixed_axis == ax && kPatchFrames[k].fixed_sign == sign) m = k;
      const PatchFrame &f = kPatchFrames[m];
      const double a = X[f.a_axis] / den, b = X[f.b_axis] / den;
      patch[i] = m;
      st[2 * i] = (a + 1.0) / 2.0;
      st[2 * i + 1] = (b + 1.0) / 2.0;
    }
  });
}

gf_status gf_space_create(gf_context *ctx, const gf_geometry *geom, int32_t degree, int32_t level, int32_t nquad,
                          int32_t mg_levels, gf_space **out) {
  return guarded([&] {
    if (!ctx || !geom || !out) fail(GF_EINVAL, "null argument");
    *out = nullptr;
    if (degree < 1 || degree > 5) fail(GF_EINVAL, "degree must be in 1..5");
    if (level < 0 || level > 12) fail(GF_EINVAL, "level must be in 0..12");
    if (nquad == 0) nquad = degree + 1;
    if (nquad < degree + 1) fail(GF_EINVAL, "nquad must be 0 or at least degree + 1");
    if (nquad > degree + 2) fail(GF_EUNSUPPORTED, "nquad above degree + 2 is not supported");
    if (mg_levels < 0 || mg_levels > level + 1) fail(GF_EINVAL, "mg_levels must be in 0..level+1");
    const int lc = mg_levels == 0 ? 0 : level + 1 - mg_levels;
    HIPCHK(hipSetDevice(ctx->device));
    std::unique_ptr<gf_space> sp(new gf_space());
    sp->ctx = ctx;
    sp->geom = const_cast<gf_geometry *>(geom);
    sp->p = degree;
    sp->j = level;
    sp->q = nquad;
    sp->lc = lc;
    // the surface for the metric kernel; NURBS control nets on the device while the levels are built
    SurfaceArgs surf;
    surf.kind = geom->kind;
    surf.amp = geom->amp;
    surf.npatch = geom->npatch;
    DBuf<int> d_pinfo;
    DBuf<double> d_knots, d_ctrl;
    if (geom->kind == SURF_NURBS) {
      d_pinfo.upload(geom->nurbs.pinfo, ctx->stream);
      d_knots.upload(geom->nurbs.knots, ctx->stream);
      d_ctrl.upload(geom->nurbs.ctrl, ctx->stream);
      surf.du = geom->nurbs.du;
      surf.dv = geom->nurbs.dv;
      surf.pinfo = d_pinfo.p;
      surf.knots = d_knots.p;
      surf.ctrl = d_ctrl.p;
    }
    for (int l = lc; l <= level; ++l) {
      std::unique_ptr<Level> L(new Level());
      build_level_host(*L, degree, l, nquad, geom);
      build_level_device(sp.get(), *L, surf);
      sp->lev.push_back(std::move(L));
    }
    for (int i = 1; i < sp->nlev(); ++i) build_transfer(sp.get(), *sp->lev[i], *sp->lev[i - 1]);
    build_coarse_dense(sp.get());
    sp->geom->refs++;
    *out = sp.release();
  });
}

void gf_space_destroy(gf_space *sp) {
  if (!sp) return;
  drop_graphs_of(sp->ctx, sp);
  ws_registry().erase(sp);
  gf_geometry_destroy(sp->geom);
  delete sp;
}

int64_t gf_space_ndofs(const gf_space *sp) { return sp ? (int64_t)sp->lev.back()->N : -1; }

int64_t gf_space_noise_length(const gf_space *sp) {
  if (!sp) return -1;
  return (int64_t)sp->fine().npatch * (int64_t)(1 << sp->j) * (int64_t)(1 << sp->j) * (sp->p + 1) * (sp->p + 1);
}

gf_status gf_space_dofmap(const gf_space *sp, int32_t *l2g) {
  return guarded([&] {
    if (!sp || !l2g) fail(GF_EINVAL, "null argument");
    const Level &F = *sp->lev.back();
    std::memcpy(l2g, F.l2g.data(), F.l2g.size() * sizeof(int32_t));
  });
}

// device copy of a caller array (or the caller's device pointer itself)
struct InArray {
  const double *p = nullptr;
  DBuf<double> own;
};
static void stage_in(InArray &a, const double *src, size_t n, int mem, hipStream_t s) {
  if (mem == GF_DEVICE) {
    a.p = src;
  } else {
    a.own.upload(src, n, s);
    a.p = a.own.p;
  }
}
struct OutArray {
  double *p = nullptr;
  double *host = nullptr;
  size_t n = 0;
  DBuf<double> own;
};
static void stage_out(OutArray &a, double *dst, size_t n, int mem) {
  a.n = n;
  if (mem == GF_DEVICE) {
    a.p = dst;
  } else {
    a.own.alloc(n);
    a.p = a.own.p;
    a.host = dst;
  }
}
static void finish_out(OutArray &a, hipStream_t s) {
  if (a.host) HIPCHK(hipMemcpyAsync(a.host, a.p, a.n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

gf_status gf_space_apply(const gf_space *csp, double sigma, double s_scale, int32_t nvec, const double *x, double *y,
                         int32_t mem, int32_t kind) {
  return guarded([&] {
    gf_space *sp = const_cast<gf_space *>(csp);
    if (!sp || !x || !y) fail(GF_EINVAL, "null argument");
    if (nvec < 1) fail(GF_EINVAL, "nvec must be >= 1");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    if (kind != GF_APPLY_STENCIL && kind != GF_APPLY_SUMFACT) fail(GF_EINVAL, "unknown operator kind");
    if (!std::isfinite(sigma) || !std::isfinite(s_scale)) fail(GF_EINVAL, "sigma and s_scale must be finite");
    HIPCHK(hipSetDevice(sp->ctx->device));
    hipStream_t s = sp->ctx->stream;
    const Level &F = sp->fine();
    const size_t n = (size_t)nvec * F.N;
    InArray xin;
    stage_in(xin, x, n, mem, s);
    OutArray yout;
    stage_out(yout, y, n, mem);
    const int ldb = round_up(nvec, CT), nt = ldb / CT;
    DBuf<double> X, Y, ca, cb;
    X.alloc((size_t)F.R * ldb);
    Y.alloc((size_t)F.R * ldb);
    ca.upload(std::vector<double>(ldb, sigma), s);
    cb.upload(std::vector<double>(ldb, s_scale), s);
    global_to_local(F, X.p, xin.p, nvec, ldb, s);
    apply_level<double>(F, kind, X.p, Y.p, ca.p, cb.p, ldb, nt, nullptr, s);
    local_to_global(F, yout.p, Y.p, nvec, 0, ldb, s);
    finish_out(yout, s);
  });
}

gf_status gf_space_apply_noalloc(const gf_space *csp, double sigma, double s_scale, int32_t nvec, const double *x,
                                 double *y, int32_t kind) {
  return guarded([&] {
    gf_space *sp = const_cast<gf_space *>(csp);
    if (!sp || !x || !y) fail(GF_EINVAL, "null argument");
    if (nvec < 1) fail(GF_EINVAL, "nvec must be >= 1");
    if (kind != GF_APPLY_STENCIL && kind != GF_APPLY_SUMFACT) fail(GF_EINVAL, "unknown operator kind");
    if (!std::isfinite(sigma) || !std::isfinite(s_scale)) fail(GF_EINVAL, "sigma and s_scale must be finite");
    const Level &F = sp->fine();
    const int ldb = round_up(nvec, CT), nt = ldb / CT;
    const size_t need = 2 * (size_t)F.R * ldb + 2 * (size_t)ldb;
    if (need * sizeof(double) > kNoAllocBytes) {
      std::ostringstream os;
      os << "nvec " << nvec << " needs " << need * sizeof(double) << " bytes of work space on this space; the "
         << "allocation-free apply has " << kNoAllocBytes << " (at most "
         << (kNoAllocBytes / sizeof(double) - 2 * CT) / (2 * (size_t)F.R + 2) / CT * CT << " vectors)";
      fail(GF_EINVAL, os.str());
    }
    HIPCHK(hipSetDevice(sp->ctx->device));
    double *base = noalloc_scratch(sp->ctx->device);
    if (!base) fail(GF_EDEVICE, "allocation-free work space not registered for this device");
    hipStream_t s = sp->ctx->stream;
    double *X = base, *Y = base + (size_t)F.R * ldb, *ca = Y + (size_t)F.R * ldb, *cb = ca + ldb;
    hipLaunchKernelGGL(k_fill2, dim3((ldb + 255) / 256), dim3(256), 0, s, ca, sigma, cb, s_scale, ldb);
    HIPCHK(hipGetLastError());
    global_to_local(F, X, x, nvec, ldb, s);
    if (kind == GF_APPLY_SUMFACT) {
      launch_sumfact_apply<double>(F, X, Y, ca, cb, ldb, nt, nullptr, s);
      launch_interface_sum<double>(F, Y, ldb, nt, nullptr, s);
    } else {
      // a fixed launch shape: the autotuner would time candidates into buffers of its own
      ApplyTune t;
      t.TY = 2;
      t.TX = 32;
      EpiArgs<double> e;
      e.kind = EPI_STORE;
      e.y = Y;
      e.nslot = 1;
      e.rows16 = 1;
      Scratch none;
      apply_fused<double>(F, F.stM.p, F.stS.p, X, ca, cb, e, none, nullptr, nullptr, ldb, nt, 0.0, 0, s, t);
    }
    local_to_global(F, y, Y, nvec, 0, ldb, s);
  });
}

gf_status gf_space_transfer(const gf_space *csp, int32_t level, int32_t direction, int32_t nvec, const double *x,
                            double *y, int32_t mem) {
  return guarded([&] {
    gf_space *sp = const_cast<gf_space *>(csp);
    if (!sp || !x || !y) fail(GF_EINVAL, "null argument");
    if (nvec < 1) fail(GF_EINVAL, "nvec must be >= 1");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    if (direction != GF_PROLONG && direction != GF_RESTRICT) fail(GF_EINVAL, "unknown direction");
    const int li = level - sp->lc;  // index of the finer level in the hierarchy
    if (li < 1 || li >= sp->nlev()) fail(GF_EINVAL, "level must be in lc+1 .. the space's level");
    HIPCHK(hipSetDevice(sp->ctx->device));
    hipStream_t s = sp->ctx->stream;
    const Level &F = *sp->lev[li], &C = *sp->lev[li - 1];
    const Level &In = direction == GF_PROLONG ? C : F, &Out = direction == GF_PROLONG ? F : C;
    InArray xin;
    stage_in(xin, x, (size_t)nvec * In.N, mem, s);
    OutArray yout;
    stage_out(yout, y, (size_t)nvec * Out.N, mem);
    const int ldb = round_up(nvec, CT), nt = ldb / CT;
    DBuf<double> XL, YL;  // patch-local layouts, zero-filled (ghost rows stay zero)
    XL.alloc((size_t)In.R * ldb);
    YL.alloc((size_t)Out.R * ldb);
    global_to_local(In, XL.p, xin.p, nvec, ldb, s);  // every copy of an unknown holds its value
    if (direction == GF_PROLONG) {
      prolong_add<double>(F, C, YL.p, XL.p, ldb, nt, nullptr, s);
    } else {
      // each fine unknown contributes once (owner copies), per patch; the coarse copies are summed
      restrict_residual<double>(F, C, YL.p, XL.p, nullptr, ldb, nt, nullptr, s);
      launch_interface_sum<double>(C, YL.p, ldb, nt, nullptr, s);
    }
    local_to_global(Out, yout.p, YL.p, nvec, 0, ldb, s);
    finish_out(yout, s);
  });
}

gf_status gf_space_cache_info(const gf_space *sp, int32_t *nplans, int64_t *plan_bytes, int32_t *nworkspaces,
                              int64_t *workspace_bytes) {
  return guarded([&] {
    if (!sp) fail(GF_EINVAL, "null argument");
    int64_t pb = 0, wb = 0;
    for (const auto &kv : sp->plans) pb += (int64_t)(kv.second->Ainv.n * sizeof(double));
    int32_t nw = 0;
    auto reg = ws_registry().find(sp);
    if (reg != ws_registry().end() && reg->second)
      for (const auto &kv : reg->second->m) {
        wb += (int64_t)kv.second->bytes;
        ++nw;
      }
    if (nplans) *nplans = (int32_t)sp->plans.size();
    if (plan_bytes) *plan_bytes = pb;
    if (nworkspaces) *nworkspaces = nw;
    if (workspace_bytes) *workspace_bytes = wb;
  });
}

gf_status gf_white_noise(const gf_space *csp, int32_t nsamp, const double *z, double *b, int32_t mem) {
  return guarded([&] {
    gf_space *sp = const_cast<gf_space *>(csp);
    if (!sp || !z || !b) fail(GF_EINVAL, "null argument");
    if (nsamp < 1) fail(GF_EINVAL, "nsamp must be >= 1");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    HIPCHK(hipSetDevice(sp->ctx->device));
    hipStream_t s = sp->ctx->stream;
    const Level &F = sp->fine();
    const size_t nz = (size_t)nsamp * gf_space_noise_length(sp);
    InArray zin;
    stage_in(zin, z, nz, mem, s);
    OutArray bout;
    stage_out(bout, b, (size_t)nsamp * F.N, mem);
    DBuf<double> ye, BL;
    ye.alloc(nz);
    const int ldb = round_up(nsamp, CT);
    BL.alloc((size_t)F.R * ldb);
    launch_white_noise(F, zin.p, nsamp, ye.p, BL.p, ldb, s);
    // interface sum of the per-patch contributions, then owner copies out
    launch_interface_sum<double>(F, BL.p, ldb, ldb / CT, nullptr, s);
    local_to_global(F, bout.p, BL.p, nsamp, 0, ldb, s);
    finish_out(bout, s);
  });
}

static void check_common(gf_space *sp, double kappa, double beta, const gf_quad_rule *rule,
                         const gf_solve_opts *opts, int32_t nsamp, int32_t mem) {
  if (!sp || !rule || !opts) fail(GF_EINVAL, "null argument");
  if (rule->split != GF_SPLIT_PLAIN && rule->split != GF_SPLIT_IMPROVED) fail(GF_EINVAL, "unknown split");
  if (!(kappa > 0.0) || !std::isfinite(kappa)) fail(GF_EINVAL, "kappa must be positive and finite");
  if (!(beta > 0.0) || !std::isfinite(beta) || beta > 64.0) fail(GF_EINVAL, "beta must be in (0, 64]");
  if (!(rule->h > 0.0) || !std::isfinite(rule->h) || rule->k_minus < 0 || rule->k_plus < 0)
    fail(GF_EINVAL, "quadrature rule needs h > 0 and k_minus, k_plus >= 0");
  if (opts->precision != GF_PREC_FP64 && opts->precision != GF_PREC_MIXED) fail(GF_EINVAL, "unknown precision");
  if (!(opts->rtol > 0.0) || !(opts->rtol < 1.0)) fail(GF_EINVAL, "rtol must be in (0, 1)");
  if (opts->max_iter < 1) fail(GF_EINVAL, "max_iter must be >= 1");
  if (opts->cheb_degree < 0 || opts->cheb_degree > 16) fail(GF_EINVAL, "cheb_degree must be in 0..16");
  if (opts->apply_kind != GF_APPLY_STENCIL && opts->apply_kind != GF_APPLY_SUMFACT)
    fail(GF_EINVAL, "unknown apply_kind");
  if (opts->preconditioner != GF_PRECOND_VCYCLE && opts->preconditioner != GF_PRECOND_BPX)
    fail(GF_EINVAL, "unknown preconditioner");
  if (nsamp < 1) fail(GF_EINVAL, "nsamp must be >= 1");
  if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
}

}  // extern "C"

namespace gf {

// beta = n + passes * bf: the plain split n = floor(beta), bf = beta - n, one pass; or the improved
// split of Sec. 3.4: bf < 1/3 (and n >= 1) -> n-1 integer solves and the rule for (bf+1)/2 twice;
// bf > 2/3 -> n integer solves and the rule for bf/2 twice
static void split_beta(double beta, int mode, int *n, double *bf, int *passes) {
  *n = (int)std::floor(beta);
  *bf = beta - *n;
  *passes = 1;
  if (mode != GF_SPLIT_IMPROVED) return;
  if (*bf > 0.0 && *bf < 1.0 / 3.0 && *n >= 1) {
    *n -= 1;
    *bf = (*bf + 1.0) / 2.0;
    *passes = 2;
  } else if (*bf > 2.0 / 3.0) {
    *bf /= 2.0;
    *passes = 2;
  }
}

// One sampling request: a space, kappa, beta, a node rule and nsamp loads.
struct SampleItem {
  gf_space *sp = nullptr;
  double kappa = 0, beta = 0;
  gf_quad_rule rule{};
  int nsamp = 0;
  const double *b = nullptr;
  double *u = nullptr;
  gf_tape *tape = nullptr;  // when set, the solutions are saved for the adjoint
  // derived
  int n = 0;       // integer solves
  double bf = 0;   // order of the sinc rule
  int passes = 1;  // applications of the rule (2 for the improved split)
  std::vector<double> node_sig, omega;
  const Plan *chain_plan = nullptr, *frac_plan = nullptr;
  InArray bin;
  OutArray uout;
  DBuf<double> rloc;
  Workspace *wc = nullptr, *wf = nullptr;
};

// All requests advance together: the integer chains step by step (step i batches every request with
// n >= i), then the sinc-node batches of all requests in one graph.  Fields are summed per request.
static void run_items(gf_context *ctx, std::vector<SampleItem> &items, const gf_solve_opts *opts, int32_t mem,
                      gf_solve_stats *stats) {
  hipStream_t s = ctx->stream;
  {
    std::vector<gf_space *> seen;
    for (auto &it : items)
      if (std::find(seen.begin(), seen.end(), it.sp) == seen.end()) {
        seen.push_back(it.sp);
        begin_call(it.sp);
      }
  }
  SolveSpec base;
  base.prec = opts->precision;
  base.kind = opts->apply_kind;
  base.cheb = opts->cheb_degree > 0 ? opts->cheb_degree : kDefaultCheb;
  base.cheb_auto = opts->cheb_degree <= 0;
  base.rtol = opts->rtol;
  base.max_iter = opts->max_iter;
  base.flags = opts->flags;
  base.precond = opts->preconditioner;
  const bool any_frac = std::any_of(items.begin(), items.end(), [](const SampleItem &it) {
    return it.beta - std::floor(it.beta) > 0.0;
  });
  // plans (their set-up is reported separately)
  double setup_ms = 0.0;
  {
    auto c0 = std::chrono::steady_clock::now();
    bool built = false;
    for (auto &it : items) {
      const size_t np = it.sp->plans.size();
      split_beta(it.beta, it.rule.split, &it.n, &it.bf, &it.passes);
      if (it.n > 0) it.chain_plan = &get_plan(it.sp, std::vector<double>{it.kappa * it.kappa});
      if (it.bf > 0.0) {
        for (int k = -it.rule.k_minus; k <= it.rule.k_plus; ++k) {
          const double t = std::exp(-2.0 * k * it.rule.h);
          it.node_sig.push_back(it.kappa * it.kappa + t);
          it.omega.push_back(2.0 * it.rule.h * std::sin(M_PI * it.bf) / M_PI * std::pow(t, 1.0 - it.bf));
        }
        it.frac_plan = &get_plan(it.sp, it.node_sig);
      }
      built = built || it.sp->plans.size() != np;
    }
    if (built) setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
  }
  // requests on one space with the same rule and split share one node batch (their columns side by
  // side, each with its own shift, under one plan for the union of their shifts); a request with a
  // tape keeps a batch of its own
  struct NodeGroup {
    gf_space *sp = nullptr;
    std::vector<SampleItem *> its;
    std::vector<int> off;  // first column of each request
    int ncols = 0;
    const Plan *plan = nullptr;
  };
  std::vector<NodeGroup> groups;
  {
    auto c0 = std::chrono::steady_clock::now();
    bool built = false;
    for (auto &it : items) {
      if (it.bf <= 0.0) continue;
      int gi = -1;
      if (!it.tape)
        for (size_t q = 0; q < groups.size(); ++q) {
          const SampleItem &h = *groups[q].its[0];
          if (groups[q].sp == it.sp && !h.tape && h.n == it.n && h.bf == it.bf && h.passes == it.passes &&
              h.omega == it.omega) {
            gi = (int)q;
            break;
          }
        }
      if (gi < 0) {
        groups.emplace_back();
        groups.back().sp = it.sp;
        gi = (int)groups.size() - 1;
      }
      NodeGroup &gr = groups[gi];
      gr.its.push_back(&it);
      gr.off.push_back(gr.ncols);
      gr.ncols += (int)it.node_sig.size() * it.nsamp;
    }
    for (auto &gr : groups) {
      if (gr.its.size() == 1) {
        gr.plan = gr.its[0]->frac_plan;
        continue;
      }
      std::vector<double> usig;
      for (auto *it : gr.its) usig.insert(usig.end(), it->node_sig.begin(), it->node_sig.end());
      const size_t np = gr.sp->plans.size();
      gr.plan = &get_plan(gr.sp, usig);
      built = built || gr.sp->plans.size() != np;
    }
    if (built) setup_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
  }
  for (auto &it : items) {
    const size_t nv = (size_t)it.nsamp * it.sp->fine().N;
    stage_in(it.bin, it.b, nv, mem, s);
    stage_out(it.uout, it.u, nv, mem);
  }
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, s));
  const int64_t sync0 = ctx->host_syncs;
  int max_it = 0, flags = 0, nsys = 0;
  double max_rel = 0.0, apply_ms = 0.0, apply_col_sum = 0.0, apply_bytes = 0.0, smooth_ms = 0.0, smooth_bytes = 0.0;
  int smooth_launches = 0;
  int apply_launches = 0, apply_rows = 0;
  auto account = [&](const BatchSolve &b) {
    max_it = std::max(max_it, b.res.max_it);
    max_rel = std::max(max_rel, b.res.max_rel);
    flags |= b.res.flags;
    nsys += b.spec.ncols;
    apply_ms += b.res.apply_ms;
    apply_launches += b.res.apply_launches;
    apply_col_sum += b.res.apply_col_sum;
    apply_bytes += b.res.apply_bytes;
    smooth_ms += b.res.smooth_ms;
    smooth_launches += b.res.smooth_launches;
    smooth_bytes += b.res.smooth_bytes;
    if (b.res.apply_launches) apply_rows = b.sp->fine().npatch * b.sp->fine().n1 * b.sp->fine().n1;
  };
  const bool use_graph = !(base.flags & (GF_FLAG_NO_GRAPH | GF_FLAG_TIME_APPLY));
  // ---- integer chains: A w_1 = b, A w_i = M w_{i-1}
  int max_n = 0;
  for (auto &it : items) max_n = std::max(max_n, it.n);
  for (size_t idx = 0; idx < items.size(); ++idx) {
    auto &it = items[idx];
    if (it.n == 0) continue;
    const Level &F = it.sp->fine();
    const int ldc = round_up(it.nsamp, CT);
    it.wc = &get_workspace(it.sp, ldc, base.prec, (int)idx);
    global_to_local(F, it.wc->r.p, it.bin.p, it.nsamp, ldc, s);
  }
  for (int i = 1; i <= max_n; ++i) {
    std::vector<BatchSolve> bs;
    bs.reserve(items.size());
    for (auto &it : items) {
      if (it.n < i) continue;
      BatchSolve b;
      b.sp = it.sp;
      b.w = it.wc;
      b.spec = base;
      if (any_frac) b.spec.flags &= ~GF_FLAG_TIME_APPLY;  // the node batches are timed instead
      b.spec.ncols = it.nsamp;
      b.spec.col_sig.assign(it.nsamp, it.kappa * it.kappa);
      b.spec.col_node.assign(it.nsamp, 0);
      b.spec.plan = it.chain_plan;
      bs.push_back(std::move(b));
    }
    std::vector<BatchSolve *> ptrs;
    for (auto &b : bs) ptrs.push_back(&b);
    solve_all(ctx, ptrs, use_graph);
    for (auto &b : bs) account(b);
    for (auto &it : items) {
      if (it.n < i) continue;
      const Level &F = it.sp->fine();
      const int ldc = it.wc->ldb;
      if (it.tape) {
        DBuf<double> &dst = it.tape->w[i - 1];
        dst.alloc((size_t)F.R * ldc);
        HIPCHK(hipMemcpyAsync(dst.p, it.wc->x.p, (size_t)F.R * ldc * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      if (i < it.n || it.bf > 0.0)  // next right-hand side M w_i (assembled)
        apply_level<double>(F, GF_APPLY_STENCIL, it.wc->x.p, it.wc->r.p, it.wc->one64.p, it.wc->zero64.p, ldc,
                            ldc / CT, nullptr, s);
      if (i == it.n && it.bf == 0.0) local_to_global(F, it.uout.p, it.wc->x.p, it.nsamp, 0, ldc, s);
    }
  }
  // ---- sinc nodes: all nodes x samples of every request, one batch per group of requests, one graph.  The
  // improved split applies the rule a second time, to M times the first result.
  int max_pass = 0;
  for (auto &it : items)
    if (it.bf > 0.0) max_pass = std::max(max_pass, it.passes);
  for (int pass = 0; pass < max_pass; ++pass) {
    std::vector<BatchSolve> bs;
    std::vector<NodeGroup *> owners;
    bs.reserve(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      NodeGroup &gr = groups[gi];
      if (pass >= gr.its[0]->passes) continue;
      const Level &F = gr.sp->fine();
      const int ldf = round_up(gr.ncols, CT);
      Workspace *wf = &get_workspace(gr.sp, ldf, base.prec, 1000 + (int)gi);
      BatchSolve b;
      b.sp = gr.sp;
      b.w = wf;
      b.spec = base;
      b.spec.ncols = gr.ncols;
      b.spec.col_sig.resize(gr.ncols);
      b.spec.col_node.resize(gr.ncols);
      int node0 = 0;  // first node of the request in the group's plan
      for (size_t q = 0; q < gr.its.size(); ++q) {
        SampleItem &it = *gr.its[q];
        const int K = (int)it.node_sig.size();
        const int ldc = round_up(it.nsamp, CT);
        const double *rsrc;
        int ldr;
        if (pass > 0) {
          rsrc = it.rloc.p;  // M v of the previous pass
          ldr = ldc;
        } else if (it.n > 0) {
          rsrc = it.wc->r.p;
          ldr = it.wc->ldb;
        } else {
          it.rloc.alloc((size_t)F.R * ldc);
          global_to_local(F, it.rloc.p, it.bin.p, it.nsamp, ldc, s);
          rsrc = it.rloc.p;
          ldr = ldc;
        }
        it.wf = wf;
        // this request's K nsamp columns only: the writes stay inside its column range
        replicate_cols(F, wf->r.p + gr.off[q], ldf, rsrc, ldr, it.nsamp, K, s, K * it.nsamp);
        for (int k = 0; k < K; ++k)
          for (int sm = 0; sm < it.nsamp; ++sm) {
            b.spec.col_sig[gr.off[q] + k * it.nsamp + sm] = it.node_sig[k];
            b.spec.col_node[gr.off[q] + k * it.nsamp + sm] = node0 + k;
          }
        node0 += K;
      }
      if (ldf > gr.ncols)  // zero padding columns after the last request
        replicate_cols(F, wf->r.p + gr.ncols, ldf, nullptr, 0, 1, 0, s, ldf - gr.ncols);
      const SampleItem &h = *gr.its[0];
      b.spec.plan = gr.plan;
      b.spec.smooth_load = h.n + pass * h.bf >= 1.5;
      bs.push_back(std::move(b));
      owners.push_back(&gr);
    }
    if (bs.empty()) continue;
    std::vector<BatchSolve *> ptrs;
    for (auto &b : bs) ptrs.push_back(&b);
    solve_all(ctx, ptrs, use_graph);
    for (size_t q = 0; q < bs.size(); ++q) {
      account(bs[q]);
      NodeGroup &gr = *owners[q];
      for (size_t m = 0; m < gr.its.size(); ++m) {
        SampleItem &it = *gr.its[m];
        const Level &F = it.sp->fine();
        if (it.tape) {  // alone in its group: the node solutions start at column 0
          const size_t nx = (size_t)F.R * it.wf->ldb;
          if ((int)it.tape->xk.size() < it.passes) it.tape->xk.resize(it.passes);
          it.tape->xk[pass].alloc(nx);
          HIPCHK(hipMemcpyAsync(it.tape->xk[pass].p, it.wf->x.p, nx * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        DBuf<double> om;
        om.upload(it.omega, s);
        // the sum lands in u; before a further pass it becomes that pass's right-hand side M u
        quadrature_sum(F, it.uout.p, it.wf->x.p + gr.off[m], om.p, (int)it.omega.size(), it.nsamp, it.wf->ldb, s);
        if (pass + 1 < it.passes) {
          const int ldc = round_up(it.nsamp, CT);
          DBuf<double> vloc;
          vloc.alloc((size_t)F.R * ldc);
          global_to_local(F, vloc.p, it.uout.p, it.nsamp, ldc, s);
          it.rloc.alloc((size_t)F.R * ldc);
          Workspace &wv = *it.wf;
          apply_level<double>(F, GF_APPLY_STENCIL, vloc.p, it.rloc.p, wv.one64.p, wv.zero64.p, ldc, ldc / CT, nullptr,
                              s);
          HIPCHK(hipStreamSynchronize(s));  // before vloc is released
        }
        HIPCHK(hipStreamSynchronize(s));
      }
    }
  }
  HIPCHK(hipEventRecord(t1, s));
  for (auto &it : items) finish_out(it.uout, s);
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (stats) {
    stats->n_systems = nsys;
    stats->max_iters = max_it;
    stats->max_rel_resid = max_rel;
    stats->setup_ms = setup_ms;
    stats->solve_ms = ms;
    stats->apply_ms = apply_ms;
    stats->apply_launches = apply_launches;
    stats->apply_rows = apply_rows;
    stats->apply_col_sum = apply_col_sum;
    stats->apply_bytes = apply_bytes;
    stats->smooth_ms = smooth_ms;
    stats->smooth_launches = smooth_launches;
    stats->smooth_bytes = smooth_bytes;
    stats->host_syncs = (int32_t)(ctx->host_syncs - sync0);
  }
  if (flags & 2) fail(GF_EBREAKDOWN, "conjugate gradients broke down in some system");
  if (flags & 1) fail(GF_ENOCONV, "some system did not reach rtol within max_iter");
}

// d L_s / d kappa for every sample s from dL/du_s = g_s and a tape of the forward solve (Sec. 3.4
// differentiated in kappa; omega_k and t_k do not depend on kappa, sigma_k = kappa^2 + t_k, and every
// matrix is symmetric):
//   lambda_{k,s} = (sigma_k M + S)^-1 g_s                          (one batch: all nodes x samples)
//   term_s  = sum_k omega_k lambda_{k,s}^T M x_{k,s}
//   mu_s    = sum_k omega_k lambda_{k,s};   nu_n = A^-1 M mu  (nu_n = A^-1 g if beta is an integer)
//   nu_{i-1} = A^-1 M nu_i,   term_s += sum_i nu_{i,s}^T M w_{i,s},     A = kappa^2 M + S
//   dL_s/dkappa = -2 kappa term_s
// The adjoint systems are solved by the same batched MG-PCG as the forward ones.
static void run_grad(gf_tape &t, const double *g_in, double *grad, int mem, gf_solve_stats *stats) {
  gf_space *sp = t.sp;
  gf_context *ctx = sp->ctx;
  hipStream_t s = ctx->stream;
  const Level &F = sp->fine();
  const int nsamp = t.nsamp;
  const int K = (int)t.node_sig.size();
  SolveSpec base;
  base.prec = t.opts.precision;
  base.kind = t.opts.apply_kind;
  base.cheb = t.opts.cheb_degree > 0 ? t.opts.cheb_degree : kDefaultCheb;
  base.cheb_auto = t.opts.cheb_degree <= 0;
  base.rtol = t.opts.rtol;
  base.max_iter = t.opts.max_iter;
  base.flags = t.opts.flags;
  base.precond = t.opts.preconditioner;
  const bool use_graph = !(base.flags & (GF_FLAG_NO_GRAPH | GF_FLAG_TIME_APPLY));
  double setup_ms = 0.0;
  const Plan *chain_plan = nullptr, *frac_plan = nullptr;
  {
    const size_t np = sp->plans.size();
    auto c0 = std::chrono::steady_clock::now();
    if (t.n > 0) chain_plan = &get_plan(sp, std::vector<double>{t.kappa * t.kappa});
    if (t.bf > 0.0) frac_plan = &get_plan(sp, t.node_sig);
    if (sp->plans.size() != np)
      setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
  }
  InArray gin;
  stage_in(gin, g_in, (size_t)nsamp * F.N, mem, s);
  OutArray gout;
  stage_out(gout, grad, (size_t)nsamp, mem);
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, s));
  const int64_t sync0 = ctx->host_syncs;
  DBuf<double> acc, dots, one;
  acc.alloc(nsamp);
  dots.alloc((size_t)2 * std::max(t.ldf, t.ldc));
  one.upload(std::vector<double>{1.0}, s);
  SolveResult tot;
  int nsys = 0;
  auto account = [&](const BatchSolve &b) {
    tot.max_it = std::max(tot.max_it, b.res.max_it);
    tot.max_rel = std::max(tot.max_rel, b.res.max_rel);
    tot.flags |= b.res.flags;
    tot.apply_ms += b.res.apply_ms;
    tot.apply_launches += b.res.apply_launches;
    tot.apply_col_sum += b.res.apply_col_sum;
    tot.apply_bytes += b.res.apply_bytes;
    tot.smooth_ms += b.res.smooth_ms;
    tot.smooth_launches += b.res.smooth_launches;
    tot.smooth_bytes += b.res.smooth_bytes;
    nsys += b.spec.ncols;
  };
  Workspace *wc = t.n > 0 ? &get_workspace(sp, t.ldc, base.prec, 0) : nullptr;
  if (t.bf > 0.0) {
    // the passes of the rule backwards: the last pass takes dL/du; each earlier pass takes M times
    // the weighted sum mu of the later pass's adjoint solutions
    Workspace &wf = get_workspace(sp, t.ldf, base.prec, 1000);
    DBuf<double> gloc, mloc, mu, om;
    gloc.alloc((size_t)F.R * t.ldc);
    mu.alloc((size_t)nsamp * F.N);
    om.upload(t.omega, s);
    global_to_local(F, gloc.p, gin.p, nsamp, t.ldc, s);
    const double *load = gloc.p;
    for (int pass = t.passes - 1; pass >= 0; --pass) {
      replicate_cols(F, wf.r.p, t.ldf, load, t.ldc, nsamp, K, s);
      BatchSolve b;
      b.sp = sp;
      b.w = &wf;
      b.spec = base;
      b.spec.ncols = K * nsamp;
      b.spec.col_sig.resize(b.spec.ncols);
      b.spec.col_node.resize(b.spec.ncols);
      for (int k = 0; k < K; ++k)
        for (int sm = 0; sm < nsamp; ++sm) {
          b.spec.col_sig[k * nsamp + sm] = t.node_sig[k];
          b.spec.col_node[k * nsamp + sm] = k;
        }
      b.spec.plan = frac_plan;
      b.spec.rough_load = (pass == t.passes - 1);
      std::vector<BatchSolve *> ptrs{&b};
      solve_all(ctx, ptrs, use_graph);
      account(b);
      // lambda^T M x per column, then the omega-weighted sum over nodes
      Scratch sc = wf.scratch();
      apply_level<double>(F, GF_APPLY_STENCIL, t.xk[pass].p, wf.q.p, wf.one64.p, wf.zero64.p, t.ldf, t.ldf / CT,
                          nullptr, s);
      reduce_dot<double, double>(F, wf.x.p, wf.q.p, sc, t.ldf, t.ldf / CT, nullptr, nullptr, OP_STORE, 0.0, 0, dots.p,
                                 s);
      grad_accum(dots.p, om.p, K, nsamp, acc.p, s);
      if (pass > 0 || t.n > 0) {
        // mu = sum_k omega_k lambda_k (global numbering), then M mu: the load of the earlier pass or
        // of the chain
        quadrature_sum(F, mu.p, wf.x.p, om.p, K, nsamp, t.ldf, s);
        global_to_local(F, gloc.p, mu.p, nsamp, t.ldc, s);
        if (pass > 0) {
          mloc.alloc((size_t)F.R * t.ldc);
          apply_level<double>(F, GF_APPLY_STENCIL, gloc.p, mloc.p, wf.one64.p, wf.zero64.p, t.ldc, t.ldc / CT,
                              nullptr, s);
          load = mloc.p;
        } else {
          apply_level<double>(F, GF_APPLY_STENCIL, gloc.p, wc->r.p, wc->one64.p, wc->zero64.p, t.ldc, t.ldc / CT,
                              nullptr, s);
        }
      }
    }
    HIPCHK(hipStreamSynchronize(s));  // before gloc, mloc, mu and om are released
  } else {
    global_to_local(F, wc->r.p, gin.p, nsamp, t.ldc, s);
  }
  for (int i = t.n; i >= 1; --i) {
    BatchSolve b;
    b.sp = sp;
    b.w = wc;
    b.spec = base;
    if (t.bf > 0.0) b.spec.flags &= ~GF_FLAG_TIME_APPLY;
    b.spec.ncols = nsamp;
    b.spec.col_sig.assign(nsamp, t.kappa * t.kappa);
    b.spec.col_node.assign(nsamp, 0);
    b.spec.plan = chain_plan;
    b.spec.rough_load = (t.bf == 0.0 && i == t.n);
    std::vector<BatchSolve *> ptrs{&b};
    solve_all(ctx, ptrs, use_graph);
    account(b);
    // nu_i^T M w_i
    Scratch sc = wc->scratch();
    apply_level<double>(F, GF_APPLY_STENCIL, t.w[i - 1].p, wc->q.p, wc->one64.p, wc->zero64.p, t.ldc, t.ldc / CT,
                        nullptr, s);
    reduce_dot<double, double>(F, wc->x.p, wc->q.p, sc, t.ldc, t.ldc / CT, nullptr, nullptr, OP_STORE, 0.0, 0,
                               dots.p, s);
    grad_accum(dots.p, one.p, 1, nsamp, acc.p, s);
    if (i > 1)  // next right-hand side M nu_i
      apply_level<double>(F, GF_APPLY_STENCIL, wc->x.p, wc->r.p, wc->one64.p, wc->zero64.p, t.ldc, t.ldc / CT,
                          nullptr, s);
  }
  grad_scale(acc.p, nsamp, -2.0 * t.kappa, gout.p, s);
  HIPCHK(hipEventRecord(t1, s));
  finish_out(gout, s);
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (stats) {
    stats->n_systems = nsys;
    stats->max_iters = tot.max_it;
    stats->max_rel_resid = tot.max_rel;
    stats->setup_ms = setup_ms;
    stats->solve_ms = ms;
    stats->apply_ms = tot.apply_ms;
    stats->apply_launches = tot.apply_launches;
    stats->apply_rows = F.npatch * F.n1 * F.n1;
    stats->apply_col_sum = tot.apply_col_sum;
    stats->apply_bytes = tot.apply_bytes;
    stats->smooth_ms = tot.smooth_ms;
    stats->smooth_launches = tot.smooth_launches;
    stats->smooth_bytes = tot.smooth_bytes;
    stats->host_syncs = (int32_t)(ctx->host_syncs - sync0);
  }
  if (tot.flags & 2) fail(GF_EBREAKDOWN, "conjugate gradients broke down in some adjoint system");
  if (tot.flags & 1) fail(GF_ENOCONV, "some adjoint system did not reach rtol within max_iter");
}

// host copies of evaluation points, validated
static void check_points(const gf_space *sp, int npts, const int32_t *patch, const double *st, int mem,
                         std::vector<int32_t> &ph, std::vector<double> &sh) {
  ph.resize(npts);
  sh.resize((size_t)2 * npts);
  if (npts == 0) return;
  if (mem == GF_DEVICE) {
    HIPCHK(hipMemcpy(ph.data(), patch, npts * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(sh.data(), st, 2 * (size_t)npts * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(ph.data(), patch, npts * sizeof(int32_t));
    std::memcpy(sh.data(), st, 2 * (size_t)npts * sizeof(double));
  }
  for (int i = 0; i < npts; ++i) {
    if (ph[i] < 0 || ph[i] >= sp->fine().npatch) fail(GF_EINVAL, "patch index out of range");
    for (int c = 0; c < 2; ++c)
      if (!(sh[2 * i + c] >= 0.0 && sh[2 * i + c] <= 1.0)) fail(GF_EINVAL, "parameter (s, t) outside [0, 1]");
  }
}

static void run_eval(const gf_space *csp, int npts, const int32_t *patch, const double *st, int nvec,
                     const double *in, double *out, int mem, bool adjoint) {
  gf_space *sp = const_cast<gf_space *>(csp);
  if (!sp || (npts > 0 && (!patch || !st)) || !in || !out) fail(GF_EINVAL, "null argument");
  if (npts < 0 || nvec < 1) fail(GF_EINVAL, "npts must be >= 0 and nvec >= 1");
  if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
  HIPCHK(hipSetDevice(sp->ctx->device));
  hipStream_t s = sp->ctx->stream;
  const Level &F = sp->fine();
  std::vector<int32_t> ph;
  std::vector<double> sh;
  check_points(sp, npts, patch, st, mem, ph, sh);
  DBuf<int> pd;
  DBuf<double> sd;
  if (npts > 0) {
    pd.upload(ph, s);
    sd.upload(sh, s);
  }
  const size_t nin = (size_t)nvec * (adjoint ? npts : F.N), nout = (size_t)nvec * (adjoint ? F.N : npts);
  InArray a;
  stage_in(a, in, nin, mem, s);
  OutArray o;
  stage_out(o, out, nout, mem);
  if (adjoint) {
    // per global coefficient, the (point, basis function) entries that touch it, in ascending point
    // order: the gather then sums them in that order (no atomics, the same result on every run).  The
    // element of a point is the one the device's basis evaluation picks (floor(u nel), clamped).
    const int p = F.p, nb = p + 1, nel = F.nel, n1 = F.n1;
    std::vector<int> cnt((size_t)F.N + 1, 0);
    std::vector<int> gids((size_t)npts * nb * nb);
    for (int i = 0; i < npts; ++i) {
      const int ex = std::min(std::max((int)std::floor(sh[2 * i] * nel), 0), nel - 1);
      const int ey = std::min(std::max((int)std::floor(sh[2 * i + 1] * nel), 0), nel - 1);
      for (int aa = 0; aa < nb; ++aa)
        for (int bb = 0; bb < nb; ++bb) {
          const int gid = F.l2g[((size_t)ph[i] * n1 + ey + aa) * n1 + ex + bb];
          gids[(size_t)i * nb * nb + aa * nb + bb] = gid;
          cnt[(size_t)gid + 1] += 1;
        }
    }
    for (int gi = 0; gi < F.N; ++gi) cnt[(size_t)gi + 1] += cnt[gi];
    std::vector<int> fill(cnt.begin(), cnt.end() - 1), ent(std::max<size_t>(1, gids.size()));
    for (size_t k = 0; k < gids.size(); ++k) ent[fill[gids[k]]++] = (int)k;
    DBuf<int> dptr, dent;
    DBuf<double> w;
    dptr.upload(cnt, s);
    dent.upload(ent, s);
    w.alloc(std::max<size_t>(1, gids.size()));
    launch_eval_adjoint(F, npts, sd.p, dptr.p, dent.p, w.p, nvec, a.p, o.p, s);
    finish_out(o, s);  // synchronises before the work arrays are released
  } else {
    launch_eval(F, npts, pd.p, sd.p, nvec, a.p, o.p, s);
    finish_out(o, s);
  }
}

// The identity of the global unknowns as a patch stencil: centre coefficient 1/(number of copies)
// on every patch row, so that the interface sum gives 1 per unknown; its diagonal is 1 on patch rows
// and 0 on ghost rows (whose mass diagonal is 1).  Built for the finest level on first use.
static void ensure_identity(gf_space *sp) {
  Level &F = sp->fine();
  if (F.stI.p) return;
  hipStream_t s = sp->ctx->stream;
  const int SS = F.S * F.S, W = F.W, n1 = F.n1, p = F.p;
  std::vector<int> copies(F.N, 0);
  for (int v : F.l2g) copies[v] += 1;
  std::vector<double> st((size_t)F.R * SS, 0.0), di((size_t)F.R, 0.0);
  for (int m = 0; m < F.npatch; ++m)
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix) {
        const int64_t row = (int64_t)m * W * W + (int64_t)(iy + p) * W + (ix + p);
        const int gid = F.l2g[((size_t)m * n1 + iy) * n1 + ix];
        st[(size_t)row * SS + p * F.S + p] = 1.0 / copies[gid];
        di[row] = 1.0;
      }
  F.stI.upload(st, s);
  F.dI.upload(di, s);
}

// Nodes, weights and prefactor of the square-root rule (Sec. 3.3, eq. sqrt) for bounds lo < hi:
// q = 1 - lo/hi, t_k = (k - 1/2) K(q)/Khat, w_k^2 = lo (sn/cn)^2, a_k = dn/cn^2, c = 2 K sqrt(lo)/(pi Khat)
static void sqrt_rule(double lo, double hi, int khat, std::vector<double> &w2, std::vector<double> &a, double *c) {
  const double q = 1.0 - lo / hi;
  const double K = complete_k(q);
  w2.resize(khat);
  a.resize(khat);
  for (int k = 0; k < khat; ++k) {
    double sn, cn, dn;
    jacobi_sncndn((k + 0.5) * K / khat, q, &sn, &cn, &dn);
    w2[k] = lo * (sn / cn) * (sn / cn);
    a[k] = dn / (cn * cn);
  }
  *c = 2.0 * K * std::sqrt(lo) / (M_PI * khat);
}

// Batched CG with the Jacobi preconditioner on (M + w_c I) x_c = r_c for the columns of w.r
static BatchSolve mass_solve(gf_space *sp, Workspace &w, const std::vector<double> &shift, const gf_solve_opts *o) {
  BatchSolve b;
  b.sp = sp;
  b.w = &w;
  b.spec.prec = GF_PREC_FP64;
  b.spec.kind = GF_APPLY_STENCIL;
  b.spec.rtol = o->rtol;
  b.spec.max_iter = o->max_iter;
  b.spec.flags = o->flags;
  b.spec.mass_shift = true;
  b.spec.ncols = (int)shift.size();
  b.spec.col_sig = shift;
  b.spec.col_node.assign(shift.size(), 0);
  std::vector<BatchSolve *> ptrs{&b};
  solve_all(sp->ctx, ptrs, !(o->flags & (GF_FLAG_NO_GRAPH | GF_FLAG_TIME_APPLY)));
  return b;
}

// Bounds of the spectrum of M: hi = max row sum of M (Gershgorin; the entries of M are
// non-negative), lo = half the Rayleigh quotient after eight steps of inverse iteration.
static void mass_bounds(gf_space *sp, const gf_solve_opts *o, double *lo, double *hi) {
  Level &F = sp->fine();
  hipStream_t s = sp->ctx->stream;
  Workspace &w = get_workspace(sp, CT, GF_PREC_FP64, 4001);
  DBuf<double> ones, row, g;
  {
    std::vector<double> h((size_t)F.R * CT, 0.0);
    for (int m = 0; m < F.npatch; ++m)
      for (int iy = 0; iy < F.n1; ++iy)
        for (int ix = 0; ix < F.n1; ++ix)
          h[((size_t)m * F.W * F.W + (size_t)(iy + F.p) * F.W + (ix + F.p)) * CT] = 1.0;
    ones.upload(h, s);
  }
  row.alloc((size_t)F.R * CT);
  g.alloc((size_t)F.N);
  apply_level<double>(F, GF_APPLY_STENCIL, ones.p, row.p, w.one64.p, w.zero64.p, CT, 1, nullptr, s);
  local_to_global(F, g.p, row.p, 1, 0, CT, s);
  std::vector<double> hg(F.N);
  HIPCHK(hipMemcpyAsync(hg.data(), g.p, F.N * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *hi = *std::max_element(hg.begin(), hg.end());
  // inverse iteration v <- M^-1 v / |v| from a hashed start vector
  gf_solve_opts io = *o;
  io.rtol = 1e-8;
  io.flags = 0;
  // hashed start vector, made consistent on the copies of shared unknowns (owner copy's value)
  hash_fill(F, w.r.p, CT, 1, s);
  local_to_global(F, g.p, w.r.p, 1, 0, CT, s);
  global_to_local(F, w.r.p, g.p, 1, CT, s);
  DBuf<double> dots, Mx;
  dots.alloc(2 * CT);
  Mx.alloc((size_t)F.R * CT);
  Scratch sc = w.scratch();
  double lam = 0.0;
  for (int it = 0; it < 8; ++it) {
    mass_solve(sp, w, std::vector<double>{0.0}, &io);
    // Rayleigh quotient x^T M x / x^T x of the new iterate, then r = x / |x|
    apply_level<double>(F, GF_APPLY_STENCIL, w.x.p, Mx.p, w.one64.p, w.zero64.p, CT, 1, nullptr, s);
    reduce_dot<double, double>(F, w.x.p, Mx.p, sc, CT, 1, nullptr, nullptr, OP_STORE, 0.0, 0, dots.p, s);
    std::vector<double> h1(2);
    HIPCHK(hipMemcpyAsync(h1.data(), dots.p, sizeof(double), hipMemcpyDeviceToHost, s));
    reduce_dot<double, double>(F, w.x.p, w.x.p, sc, CT, 1, nullptr, nullptr, OP_STORE, 0.0, 0, dots.p, s);
    HIPCHK(hipMemcpyAsync(h1.data() + 1, dots.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(h1[0] > 0.0) || !(h1[1] > 0.0)) fail(GF_EDEVICE, "mass-matrix bound estimate failed");
    lam = h1[0] / h1[1];
    // r = x / |x| on every patch row: the diagonal kernel with D = |x| dI + 0 dM
    DBuf<double> nrm;
    nrm.upload(std::vector<double>(CT, std::sqrt(h1[1])), s);
    div_diag2(F, w.r.p, w.x.p, nrm.p, F.dI.p, w.zero64.p, F.dM.p, CT, 1, nullptr, s);
    HIPCHK(hipStreamSynchronize(s));  // before nrm is released
  }
  *lo = 0.5 * lam;
}

}  // namespace gf

extern "C" {

gf_status gf_sqrt_mass_rule(double lo, double hi, int32_t khat, double *w2, double *a, double *c) {
  return guarded([&] {
    if (!w2 || !a || !c) fail(GF_EINVAL, "null argument");
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) fail(GF_EINVAL, "need 0 < lo < hi, finite");
    if (khat < 1 || khat > 4096) fail(GF_EINVAL, "khat must be in 1..4096");
    std::vector<double> vw, va;
    sqrt_rule(lo, hi, khat, vw, va, c);
    std::copy(vw.begin(), vw.end(), w2);
    std::copy(va.begin(), va.end(), a);
  });
}

gf_status gf_sqrt_mass(gf_space *sp, int32_t nsamp, const double *y, double *f, int32_t khat, double lo, double hi,
                       const gf_solve_opts *opts, int32_t mem, gf_solve_stats *stats) {
  return guarded([&] {
    if (!sp || !y || !f || !opts) fail(GF_EINVAL, "null argument");
    if (nsamp < 1) fail(GF_EINVAL, "nsamp must be >= 1");
    if (khat < 1 || khat > 4096) fail(GF_EINVAL, "khat must be in 1..4096");
    if ((int64_t)khat * nsamp > (int64_t)1 << 20) fail(GF_EINVAL, "too many systems in one batch");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    if (!(opts->rtol > 0.0) || !(opts->rtol < 1.0)) fail(GF_EINVAL, "rtol must be in (0, 1)");
    if (opts->max_iter < 1) fail(GF_EINVAL, "max_iter must be >= 1");
    const bool estimate = (lo == 0.0 && hi == 0.0);
    if (!estimate && (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi))) fail(GF_EINVAL, "need 0 < lo < hi, finite");
    HIPCHK(hipSetDevice(sp->ctx->device));
    begin_call(sp);
    hipStream_t s = sp->ctx->stream;
    const Level &F = sp->fine();
    auto c0 = std::chrono::steady_clock::now();
    ensure_identity(sp);
    if (estimate) mass_bounds(sp, opts, &lo, &hi);
    std::vector<double> w2, a;
    double c = 0.0;
    sqrt_rule(lo, hi, khat, w2, a, &c);
    const double setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
    const size_t nv = (size_t)nsamp * F.N;
    InArray yin;
    stage_in(yin, y, nv, mem, s);
    OutArray fout;
    stage_out(fout, f, nv, mem);
    hipEvent_t t0, t1;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    HIPCHK(hipEventRecord(t0, s));
    const int64_t sync0 = sp->ctx->host_syncs;
    const int ldc = round_up(nsamp, CT), ncols = khat * nsamp, ldf = round_up(ncols, CT);
    DBuf<double> yl;
    yl.alloc((size_t)F.R * ldc);
    global_to_local(F, yl.p, yin.p, nsamp, ldc, s);
    Workspace &w = get_workspace(sp, ldf, GF_PREC_FP64, 4000);
    replicate_cols(F, w.r.p, ldf, yl.p, ldc, nsamp, khat, s);
    std::vector<double> shift(ncols);
    for (int k = 0; k < khat; ++k)
      for (int sm = 0; sm < nsamp; ++sm) shift[k * nsamp + sm] = w2[k];
    BatchSolve b = mass_solve(sp, w, shift, opts);
    // g = c sum_k a_k z_k (ascending k), f = M g
    std::vector<double> om(khat);
    for (int k = 0; k < khat; ++k) om[k] = c * a[k];
    DBuf<double> omd, g;
    omd.upload(om, s);
    g.alloc(nv);
    quadrature_sum(F, g.p, w.x.p, omd.p, khat, nsamp, ldf, s);
    global_to_local(F, yl.p, g.p, nsamp, ldc, s);
    apply_level<double>(F, GF_APPLY_STENCIL, yl.p, w.q.p, w.one64.p, w.zero64.p, ldc, ldc / CT, nullptr, s);
    local_to_global(F, fout.p, w.q.p, nsamp, 0, ldc, s);
    HIPCHK(hipEventRecord(t1, s));
    finish_out(fout, s);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (stats) {
      *stats = gf_solve_stats{};
      stats->n_systems = ncols;
      stats->max_iters = b.res.max_it;
      stats->max_rel_resid = b.res.max_rel;
      stats->setup_ms = setup_ms;
      stats->solve_ms = ms;
      stats->apply_ms = b.res.apply_ms;
      stats->apply_launches = b.res.apply_launches;
      stats->apply_rows = F.npatch * F.n1 * F.n1;
      stats->apply_bytes = b.res.apply_bytes;
      stats->host_syncs = (int32_t)(sp->ctx->host_syncs - sync0);
    }
    if (b.res.flags & 2) fail(GF_EBREAKDOWN, "conjugate gradients broke down in some system");
    if (b.res.flags & 1) fail(GF_ENOCONV, "some system did not reach rtol within max_iter");
  });
}

gf_status gf_sample(gf_space *sp, double kappa, double beta, const gf_quad_rule *rule, const gf_solve_opts *opts,
                    int32_t nsamp, const double *b, double *u, int32_t mem, gf_solve_stats *stats) {
  return guarded([&] {
    check_common(sp, kappa, beta, rule, opts, nsamp, mem);
    if (!b || !u) fail(GF_EINVAL, "null argument");
    const int K = rule->k_minus + rule->k_plus + 1;
    if (beta - std::floor(beta) > 0.0 && (int64_t)K * nsamp > (int64_t)1 << 20)
      fail(GF_EINVAL, "too many systems in one batch");
    HIPCHK(hipSetDevice(sp->ctx->device));
    std::vector<SampleItem> items(1);
    items[0].sp = sp;
    items[0].kappa = kappa;
    items[0].beta = beta;
    items[0].rule = *rule;
    items[0].nsamp = nsamp;
    items[0].b = b;
    items[0].u = u;
    run_items(sp->ctx, items, opts, mem, stats);
  });
}

gf_status gf_sample_batch(gf_context *ctx, int32_t nitems, const gf_batch_item *items_in, const gf_solve_opts *opts,
                          int32_t mem, gf_solve_stats *stats) {
  return guarded([&] {
    if (!ctx || !items_in || !opts) fail(GF_EINVAL, "null argument");
    if (nitems < 1 || nitems > 4096) fail(GF_EINVAL, "nitems must be in 1..4096");
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<SampleItem> items(nitems);
    for (int i = 0; i < nitems; ++i) {
      const gf_batch_item &in = items_in[i];
      check_common(in.space, in.kappa, in.beta, &in.rule, opts, in.nsamp, mem);
      if (!in.b || !in.u) fail(GF_EINVAL, "null load or field pointer in a batch item");
      if (in.space->ctx != ctx) fail(GF_EINVAL, "batch item space belongs to another context");
      const int K = in.rule.k_minus + in.rule.k_plus + 1;
      if ((int64_t)K * in.nsamp > (int64_t)1 << 20) fail(GF_EINVAL, "too many systems in one batch item");
      items[i].sp = in.space;
      items[i].kappa = in.kappa;
      items[i].beta = in.beta;
      items[i].rule = in.rule;
      items[i].nsamp = in.nsamp;
      items[i].b = in.b;
      items[i].u = in.u;
    }
    run_items(ctx, items, opts, mem, stats);
  });
}

gf_status gf_solve_shifted(gf_space *sp, int32_t nsys, const double *sigma, const double *b, double *x,
                           const gf_solve_opts *opts, int32_t mem, gf_solve_stats *stats) {
  return guarded([&] {
    if (!sp || !sigma || !b || !x || !opts) fail(GF_EINVAL, "null argument");
    if (nsys < 1 || nsys > (1 << 20)) fail(GF_EINVAL, "nsys must be in 1..2^20");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    if (opts->precision != GF_PREC_FP64 && opts->precision != GF_PREC_MIXED) fail(GF_EINVAL, "unknown precision");
    if (!(opts->rtol > 0.0) || !(opts->rtol < 1.0)) fail(GF_EINVAL, "rtol must be in (0, 1)");
    if (opts->max_iter < 1) fail(GF_EINVAL, "max_iter must be >= 1");
    if (opts->cheb_degree < 0 || opts->cheb_degree > 16) fail(GF_EINVAL, "cheb_degree must be in 0..16");
    if (opts->apply_kind != GF_APPLY_STENCIL && opts->apply_kind != GF_APPLY_SUMFACT)
      fail(GF_EINVAL, "unknown apply_kind");
    if (opts->preconditioner != GF_PRECOND_VCYCLE && opts->preconditioner != GF_PRECOND_BPX)
      fail(GF_EINVAL, "unknown preconditioner");
    const bool mass = (opts->flags & GF_FLAG_MASS_SHIFT) != 0;
    // distinct shifts in order of first appearance: one multigrid plan node each
    std::vector<double> distinct;
    std::vector<int> node(nsys);
    for (int i = 0; i < nsys; ++i) {
      if (!(mass ? sigma[i] >= 0.0 : sigma[i] > 0.0) || !std::isfinite(sigma[i]))
        fail(GF_EINVAL, mass ? "every shift must be non-negative and finite" : "every shift must be positive and finite");
      auto f = std::find(distinct.begin(), distinct.end(), sigma[i]);
      node[i] = (int)(f - distinct.begin());
      if (f == distinct.end()) distinct.push_back(sigma[i]);
    }
    if (distinct.size() > 4096) fail(GF_EINVAL, "at most 4096 distinct shifts per call");
    HIPCHK(hipSetDevice(sp->ctx->device));
    begin_call(sp);
    hipStream_t s = sp->ctx->stream;
    const Level &F = sp->fine();
    double setup_ms = 0.0;
    const Plan *plan = nullptr;
    {
      const size_t np = sp->plans.size();
      auto c0 = std::chrono::steady_clock::now();
      if (mass)
        ensure_identity(sp);
      else
        plan = &get_plan(sp, distinct);
      if (sp->plans.size() != np)
        setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
    }
    const size_t nv = (size_t)nsys * F.N;
    InArray bin;
    stage_in(bin, b, nv, mem, s);
    OutArray xout;
    stage_out(xout, x, nv, mem);
    const int ldb = round_up(nsys, CT);
    const int prec = mass ? GF_PREC_FP64 : opts->precision;
    Workspace &w = get_workspace(sp, ldb, prec, 3000);
    hipEvent_t t0, t1;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    HIPCHK(hipEventRecord(t0, s));
    const int64_t sync0 = sp->ctx->host_syncs;
    global_to_local(F, w.r.p, bin.p, nsys, ldb, s);
    SolveSpec spec;
    spec.prec = prec;
    spec.kind = mass ? GF_APPLY_STENCIL : opts->apply_kind;
    spec.cheb = opts->cheb_degree > 0 ? opts->cheb_degree : kDefaultCheb;
    spec.cheb_auto = opts->cheb_degree <= 0;
    spec.rtol = opts->rtol;
    spec.max_iter = opts->max_iter;
    spec.flags = opts->flags;
    spec.mass_shift = mass;
    spec.precond = opts->preconditioner;
    spec.ncols = nsys;
    spec.col_sig.assign(sigma, sigma + nsys);
    spec.col_node = node;
    spec.plan = plan;
    SolveResult r = solve_batch(sp, w, spec);
    local_to_global(F, xout.p, w.x.p, nsys, 0, ldb, s);
    HIPCHK(hipEventRecord(t1, s));
    finish_out(xout, s);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (stats) {
      stats->n_systems = nsys;
      stats->max_iters = r.max_it;
      stats->max_rel_resid = r.max_rel;
      stats->setup_ms = setup_ms;
      stats->solve_ms = ms;
      stats->apply_ms = r.apply_ms;
      stats->apply_launches = r.apply_launches;
      stats->apply_rows = F.npatch * F.n1 * F.n1;
      stats->apply_col_sum = r.apply_col_sum;
      stats->apply_bytes = r.apply_bytes;
      stats->smooth_ms = r.smooth_ms;
      stats->smooth_launches = r.smooth_launches;
      stats->smooth_bytes = r.smooth_bytes;
      stats->host_syncs = (int32_t)(sp->ctx->host_syncs - sync0);
    }
    if (r.flags & 2) fail(GF_EBREAKDOWN, "conjugate gradients broke down in some system");
    if (r.flags & 1) fail(GF_ENOCONV, "some system did not reach rtol within max_iter");
  });
}

gf_status gf_sample_tape(gf_space *sp, double kappa, double beta, const gf_quad_rule *rule,
                         const gf_solve_opts *opts, int32_t nsamp, const double *b, double *u, int32_t mem,
                         gf_tape **tape, gf_solve_stats *stats) {
  return guarded([&] {
    check_common(sp, kappa, beta, rule, opts, nsamp, mem);
    if (!b || !u || !tape) fail(GF_EINVAL, "null argument");
    *tape = nullptr;
    const int K = rule->k_minus + rule->k_plus + 1;
    if (beta - std::floor(beta) > 0.0 && (int64_t)K * nsamp > (int64_t)1 << 20)
      fail(GF_EINVAL, "too many systems in one batch");
    HIPCHK(hipSetDevice(sp->ctx->device));
    std::unique_ptr<gf_tape> t(new gf_tape());
    t->sp = sp;
    t->kappa = kappa;
    t->beta = beta;
    t->rule = *rule;
    t->opts = *opts;
    t->nsamp = nsamp;
    split_beta(beta, rule->split, &t->n, &t->bf, &t->passes);
    t->ldc = round_up(nsamp, CT);
    t->ldf = round_up(K * nsamp, CT);
    t->w.resize(t->n);
    std::vector<SampleItem> items(1);
    items[0].sp = sp;
    items[0].kappa = kappa;
    items[0].beta = beta;
    items[0].rule = *rule;
    items[0].nsamp = nsamp;
    items[0].b = b;
    items[0].u = u;
    items[0].tape = t.get();
    run_items(sp->ctx, items, opts, mem, stats);
    t->node_sig = items[0].node_sig;
    t->omega = items[0].omega;
    *tape = t.release();
  });
}

gf_status gf_grad_kappa(gf_tape *tape, const double *dl_du, double *dl_dkappa, int32_t mem, gf_solve_stats *stats) {
  return guarded([&] {
    if (!tape || !dl_du || !dl_dkappa) fail(GF_EINVAL, "null argument");
    if (mem != GF_HOST && mem != GF_DEVICE) fail(GF_EINVAL, "mem must be GF_HOST or GF_DEVICE");
    HIPCHK(hipSetDevice(tape->sp->ctx->device));
    begin_call(tape->sp);
    run_grad(*tape, dl_du, dl_dkappa, mem, stats);
  });
}

void gf_tape_destroy(gf_tape *tape) { delete tape; }

gf_status gf_eval(const gf_space *space, int32_t npts, const int32_t *patch, const double *st, int32_t nvec,
                  const double *u, double *vals, int32_t mem) {
  return guarded([&] { run_eval(space, npts, patch, st, nvec, u, vals, mem, false); });
}

gf_status gf_eval_adjoint(const gf_space *space, int32_t npts, const int32_t *patch, const double *st, int32_t nvec,
                          const double *r, double *out, int32_t mem) {
  return guarded([&] { run_eval(space, npts, patch, st, nvec, r, out, mem, true); });
}

}  // extern "C"
