// Internal declarations of the gfield library: space/level data, device buffers,
// kernel launchers.  Not part of the public ABI (see include/gfield.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/gfield.h"

namespace gf {

// ------------------------------------------------------------------ errors
struct Error {
  gf_status code;
  std::string msg;
};
void set_error(const std::string &msg);
[[noreturn]] void fail(gf_status code, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPCHK(x) ::gf::hip_check((x), #x, __FILE__, __LINE__)

// ------------------------------------------------------------------ device buffer
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // (re)allocate n elements, zero-filled once at allocation
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    HIPCHK(hipMalloc((void **)&p, count * sizeof(T)));
    HIPCHK(hipMemset(p, 0, count * sizeof(T)));
    // the fill runs on the null stream: finish it before any other stream touches the buffer
    HIPCHK(hipDeviceSynchronize());
    n = count;
  }
  // copy from (pageable) host memory; returns once the copy has completed
  void upload(const T *h, size_t count, hipStream_t s) {
    alloc(count);
    HIPCHK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  void upload(const std::vector<T> &h, hipStream_t s) { upload(h.data(), h.size(), s); }
};

// ------------------------------------------------------------------ host spline helpers
struct PatchFrame {
  int fixed_axis, fixed_sign, a_axis, b_axis;
};
extern const PatchFrame kPatchFrames[6];
void gauss_legendre(int q, std::vector<double> &x, std::vector<double> &w);
void element_basis(int p, int nel, int e, double u, double *val, double *der);
std::vector<double> refinement_matrix(int p, int lc);
void glue_patches(int p, int lev, std::vector<int> &l2g, int &N);

// Description of the surface for the device (metric kernel): the six-patch sphere family, or
// rational tensor-product B-spline patches of degrees (du, dv) with, per patch, pinfo[5 m ..] =
// (control points along s, along t, offset of the s knots, offset of the t knots, offset of the
// control points) into knots[] and ctrl[] ([nt][ns][4]: x, y, z, weight).
enum SurfaceKind { SURF_SPHERE = 0, SURF_NURBS = 1 };
struct SurfaceArgs {
  int kind = SURF_SPHERE;
  double amp = 0.0;  // sphere family: amplitude of the radial perturbation (0: unit sphere)
  int npatch = 6;
  int du = 0, dv = 0;
  const int *pinfo = nullptr;
  const double *knots = nullptr;
  const double *ctrl = nullptr;
};
// host copy of a NURBS surface
struct NurbsHost {
  int npatch = 0, du = 0, dv = 0;
  std::vector<int> pinfo;
  std::vector<double> knots, ctrl;
};
// Interface gluing of the FEM coefficients of one level on NURBS patches: shared edges are found
// by comparing the boundary control points, weights and knots of the patches; coefficient rows
// along matched edges are identified (same or reversed order), corners through the edges.
void glue_patches_nurbs(const NurbsHost &g, int p, int lev, std::vector<int> &l2g, int &N);
// surface point and parameter derivatives of patch m at (s, t), on the host
void nurbs_eval(const NurbsHost &g, int m, double s, double t, double X[3], double Xs[3], double Xt[3]);
// closest point of the surface to P: patch, parameters and distance
void nurbs_locate(const NurbsHost &g, const double P[3], int *patch, double *s, double *t, double *dist);
// Jacobi elliptic functions sn, cn, dn of parameter q in [0, 1) and the complete elliptic integral
// of the first kind K(q)
void jacobi_sncndn(double u, double q, double *sn, double *cn, double *dn);
double complete_k(double q);

// launch shape of the fused stencil apply, chosen by the autotuner: TY coefficient rows per
// wavefront strip (1, 2 or 4) and at most TX coefficients along the strip
struct ApplyTune {
  int TY = 1, TX = 32, NC = 1;  // NC: 64-column tiles per wavefront
  int algo = 1;                 // 0: M and S stencils applied separately; 1: one combined stencil per
                                // distinct shift of the column tile, loads one step ahead
  int grp = 1;                  // dispatch order of the combined-stencil kernel: groups of grp
                                // vertically adjacent strip blocks per column tile (1: tiles fastest)
  float us = 0.f;               // measured duration of one launch
};

// ------------------------------------------------------------------ per-level data
// Vectors of a level live in the padded patch-local layout: patch m, coefficient (iy, ix)
// (0 <= iy, ix < n1) sits at row m*W*W + (iy+p)*W + (ix+p), W = n1 + 2p; the p ghost rows
// and columns around every patch grid are zero.  A batch of vectors is stored row-major
// with the column (system) index fastest: element (row, c) at row*ldb + c.
struct Level {
  int p = 0, lev = 0, nel = 0, n1 = 0, W = 0, q = 0, S = 0;  // S = 2p+1 stencil width
  int npatch = 6;
  int64_t R = 0;  // padded rows npatch*W*W
  int N = 0;      // unique unknowns
  std::vector<int> l2g;             // host: local (m, iy, ix) -> global id
  std::vector<int> owner_row_h;     // host: global id -> owner row
  DBuf<double> metric;              // [npatch][nel][nel][q][q][4]: m, G11, G12, G22 (weights folded in)
  DBuf<double> basis;               // [nel][2][q][p+1]: values, then s-derivatives
  DBuf<float> metric32, basis32;    // FP32 copies for the FP32 matrix-free apply
  DBuf<double> stM, stS;            // [R][S*S] patch stencils (FP64)
  DBuf<float> stM32, stS32;         // same, FP32
  DBuf<double> dM, dS;              // interface-summed diagonals [R]
  DBuf<double> stI, dI;             // identity of the global unknowns as a stencil (centre 1/copies) and its
                                    // interface-summed diagonal (1); built on first use
  DBuf<float> dM32, dS32;
  double dM_mean = 0.0, dS_mean = 0.0;  // means of dM, dS over the rows of coefficients
  DBuf<uint8_t> owner;              // [R] 1 on the owner copy of each unknown
  DBuf<int> grp_ptr, grp_rows;      // shared unknowns: CSR list of their rows
  int ngroups = 0;
  DBuf<int> owner_row;              // [N] row of the owner copy
  DBuf<int> row_gid;                // [R] global id of a row (-1 on ghosts)
  // prolongation from the next coarser level into this level (empty on level 0 of the space)
  int pw = 0, rw = 0;               // band widths of P rows / P columns
  DBuf<int> pro_start, res_start;   // per fine index: first coarse index; per coarse index: first fine index
  DBuf<double> pro_c, res_c;        // [n1f][pw], [n1c][rw]
  DBuf<float> pro_c32, res_c32;
  // autotuned launch shapes, keyed by (element size, column stride, epilogue kind, stencil mode)
  mutable std::map<std::tuple<int, int, int, int>, ApplyTune> tune;
};

}  // namespace gf

// ------------------------------------------------------------------ public handles
struct gf_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // Instantiated HIP graphs of chunks of CG iterations, by batch configuration (kept across calls; a
  // graph is dropped when a space it uses is destroyed, the least recently used beyond a bound)
  struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> events;  // the fork and join events of the capture, kept while the graph lives
    std::vector<const void *> spaces;
    uint64_t last = 0;
  };
  std::map<std::string, Graph> graphs;
  uint64_t graph_clock = 0;
  int *flag_dev = nullptr;   // 1 while some column tile of the last chunk's batches is still active
  int *flag_host = nullptr;  // its pinned host copy
  int64_t host_syncs = 0;    // host synchronisations with the stream inside CG loops (statistics)
};

struct gf_geometry {
  gf_context *ctx = nullptr;
  int kind = gf::SURF_SPHERE;
  double amp = 0.0;  // sphere family: amplitude of the radial perturbation
  int npatch = 6;
  gf::NurbsHost nurbs;                    // SURF_NURBS: the patches (host; copied to the device
                                          // while a space is built on them)
  int refs = 1;
};

namespace gf {
struct Plan;
}

struct gf_space {
  gf_context *ctx = nullptr;
  gf_geometry *geom = nullptr;
  int p = 0, j = 0, q = 0, lc = 0;
  std::vector<std::unique_ptr<gf::Level>> lev;  // lev[i] holds refinement level lc + i
  // dense coarse matrices (global numbering of level lc), FP64 on device
  gf::DBuf<double> M0, S0;
  int N0 = 0;
  std::map<std::string, std::unique_ptr<gf::Plan>> plans;
  uint64_t calls = 0;  // calls that used the space so far (recency of its cached plans and workspaces)
  // smoothing degree chosen by measurement for large batches, by batch configuration (see tune_degree)
  std::map<std::string, int> cheb_tuned;
  gf::Level &fine() { return *lev.back(); }
  const gf::Level &fine() const { return *lev.back(); }
  int nlev() const { return (int)lev.size(); }
};

namespace gf {

// ------------------------------------------------------------------ kernel launchers
// Column tiles are 64 systems wide; `active` (may be null) marks tiles still iterating.
constexpr int CT = 64;

// setup kernels (k_setup.hip)
void launch_metric(const Level &L, const SurfaceArgs &g, const double *gx, const double *gw, hipStream_t s);
template <typename T>
void launch_sumfact_apply(const Level &L, const T *x, T *y, const T *ca, const T *cb, int ldb, int ntiles,
                          const int *active, hipStream_t s);
void launch_probe_vectors(const Level &L, double *x, int ldb, hipStream_t s);
void launch_extract_stencil(const Level &L, const double *y, int ldb, double *stM, double *stS, hipStream_t s);
void launch_stencil_diag(const Level &L, hipStream_t s);

void launch_coarse_inverse(const double *Lf, int N0, int nnode, double *Ainv, hipStream_t s);
// achieved vector fused multiply-add rate in TFLOP/s (FP64 or FP32), measured on the current device
double fma_probe(bool fp64, hipStream_t s);
void launch_coarse_factor(const double *M0, const double *S0, int N0, const double *sig, int nnode, double *Lf,
                          int *info, hipStream_t s);

// solver kernels (k_solve.hip)
template <typename T>
void launch_interface_sum(const Level &L, T *y, int ldb, int ntiles, const int *active, hipStream_t s);

}  // namespace gf
