// kbench: timing of the operator kernels on one level of the six-patch layout, outside the solver
// (measurement support; links libgfield.so and calls its kernel launchers).
//
// Usage: kbench <p> <lev> <nnode> <nsamp> <f32|f64> <kinds> [algos] [shapes]
//   kinds  comma-separated: cheb (smoothing step with a previous direction), chebdot, store, storedot,
//          resid (the fused stencil kernels), sumfact (the matrix-free sum-factorised apply), copy
//          (y = -x over the whole batch: reads and writes exactly R * ldb elements; the known-size
//          reference for the memory-traffic counters)
//   algos  digits: 0 separate-stencil kernel, 1 combined-stencil kernel (default 01)
//   shapes comma-separated TY:TX or TY:TX:G launch shapes (default 1:32,2:32,1:64,2:64,4:32,4:64); G:
//          strip blocks of one column tile dispatched back to back (default: the library's)
// Columns: nnode shifts of nsamp systems each (node-major, as the sampler lays them out).  Stencils,
// metric terms and vectors are seeded pseudo-random numbers (timing does not depend on the values);
// every configuration after the first of a kind is compared with the first (relative max deviation).
// Each stencil configuration runs once per stencil mode: comb (one combined stencil per distinct
// shift of a tile), pair (separate M and S), dpp (16-lane row broadcast, when nsamp is a multiple of
// 16).  Algorithmic bytes: the batch vectors each kernel reads and writes per real row and column plus
// the two stencils per row; sum-factorised flops (20 (p+1)^3 + 8 (p+1)^2) per element and column.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2605_24882_amd/csrc/gf_internal.h"
#include "../../paper_2605_24882_amd/csrc/k_solve.h"

using namespace gf;

#define CK(x)                                                                  \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      std::fprintf(stderr, "HIP %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      std::exit(3);                                                            \
    }                                                                          \
  } while (0)

template <typename T>
__global__ void k_fill(T *v, int64_t R, int ldb, int W, int n1, int P, uint32_t seed, int real_only) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * ldb) return;
  const int64_t row = i / ldb;
  const int lx = (int)(row % W) - P, ly = (int)((row / W) % W) - P;
  const bool inside = lx >= 0 && lx < n1 && ly >= 0 && ly < n1;
  uint32_t h = (uint32_t)(i * 2654435761u) ^ seed;
  h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
  const T v0 = (T)((h & 0xffffff) / 16777216.0 - 0.5);
  v[i] = (inside || !real_only) ? v0 : T(0);
}

template <typename T>
__global__ void k_stfill(T *v, int64_t n, uint32_t seed, int SS, int centre, T cval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)(i * 2246822519u) ^ seed;
  h ^= h >> 13; h *= 0x5bd1e995u; h ^= h >> 15;
  T v0 = (T)((h & 0xffffff) / 16777216.0 - 0.5) * T(0.1);
  if ((int)(i % SS) == centre) v0 = cval;
  v[i] = v0;
}

// max |a - b| and max |b| over real rows (as bit patterns of non-negative floats)
template <typename T>
__global__ void k_cmp(const T *a, const T *b, int64_t R, int ldb, int ncols, int W, int n1, int P,
                      unsigned long long *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * ldb) return;
  const int64_t row = i / ldb;
  const int c = (int)(i % ldb);
  const int lx = (int)(row % W) - P, ly = (int)((row / W) % W) - P;
  if (!(lx >= 0 && lx < n1 && ly >= 0 && ly < n1) || c >= ncols) return;
  const double d = fabs((double)a[i] - (double)b[i]), m = fabs((double)b[i]);
  atomicMax(out, (unsigned long long)__double_as_longlong(isfinite(d) ? d : 1e300));
  atomicMax(out + 1, (unsigned long long)__double_as_longlong(m));
}

template <typename T>
__global__ void k_neg(const T *__restrict__ a, T *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

template <typename T>
static T *dalloc(size_t n) {
  T *p = nullptr;
  CK(hipMalloc((void **)&p, n * sizeof(T)));
  return p;
}

struct Shape {
  int TY, TX, G;
};

template <typename T>
static void run(int p, int lev, int nnode, int nsamp, const std::vector<std::string> &kinds,
                const std::vector<int> &algos, const std::vector<Shape> &shapes) {
  hipStream_t s = nullptr;
  Level L;
  L.p = p;
  L.lev = lev;
  L.nel = 1 << lev;
  L.n1 = L.nel + p;
  L.W = L.n1 + 2 * p;
  L.q = p + 1;
  L.S = 2 * p + 1;
  L.npatch = 6;
  L.R = (int64_t)6 * L.W * L.W;
  const int SS = L.S * L.S, W = L.W, n1 = L.n1;
  const int ncols = nnode * nsamp, ldb = (ncols + 63) / 64 * 64, nt = ldb / 64;
  std::printf("case p=%d lev=%d R=%ld rows=%d ncols=%d ldb=%d T=%s\n", p, lev, (long)L.R, 6 * n1 * n1, ncols, ldb,
              sizeof(T) == 8 ? "f64" : "f32");
  std::fflush(stdout);
  // interface groups: every patch-boundary row alone
  std::vector<int> gp{0}, gr;
  for (int m = 0; m < 6; ++m)
    for (int iy = 0; iy < n1; ++iy)
      for (int ix = 0; ix < n1; ++ix)
        if (ix == 0 || iy == 0 || ix == n1 - 1 || iy == n1 - 1) {
          gr.push_back((int)((int64_t)m * W * W + (int64_t)(iy + p) * W + ix + p));
          gp.push_back((int)gr.size());
        }
  L.ngroups = (int)gp.size() - 1;
  L.grp_ptr.upload(gp, s);
  L.grp_rows.upload(gr, s);
  const size_t nst = (size_t)L.R * SS;
  T *stM = dalloc<T>(nst), *stS = dalloc<T>(nst);
  const int centre = p * L.S + p;
  hipLaunchKernelGGL(k_stfill<T>, dim3((nst + 255) / 256), dim3(256), 0, s, stM, (int64_t)nst, 11u, SS, centre, T(1.0));
  hipLaunchKernelGGL(k_stfill<T>, dim3((nst + 255) / 256), dim3(256), 0, s, stS, (int64_t)nst, 12u, SS, centre, T(4.0));
  std::vector<T> dM(L.R), dS(L.R);
  T *ddM = dalloc<T>(L.R), *ddS = dalloc<T>(L.R);
  // diagonals = stencil centres (interior rows use these in the old kernel)
  {
    std::vector<T> h(nst);
    CK(hipMemcpy(h.data(), stM, nst * sizeof(T), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < L.R; ++r) dM[r] = h[r * SS + centre];
    CK(hipMemcpy(h.data(), stS, nst * sizeof(T), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < L.R; ++r) dS[r] = h[r * SS + centre];
    CK(hipMemcpy(ddM, dM.data(), L.R * sizeof(T), hipMemcpyHostToDevice));
    CK(hipMemcpy(ddS, dS.data(), L.R * sizeof(T), hipMemcpyHostToDevice));
  }
  // random metric terms and basis tables for the matrix-free kernel (timing only)
  {
    const int q = L.q;
    const size_t nm = (size_t)6 * L.nel * L.nel * q * q * 4, nb = (size_t)L.nel * 2 * q * (p + 1);
    if (sizeof(T) == 8) {
      L.metric.alloc(nm);
      L.basis.alloc(nb);
      hipLaunchKernelGGL(k_stfill<double>, dim3((nm + 255) / 256), dim3(256), 0, s, L.metric.p, (int64_t)nm, 21u, 4, 0, 1.0);
      hipLaunchKernelGGL(k_stfill<double>, dim3((nb + 255) / 256), dim3(256), 0, s, L.basis.p, (int64_t)nb, 22u, 1, -1, 0.0);
    } else {
      L.metric32.alloc(nm);
      L.basis32.alloc(nb);
      hipLaunchKernelGGL(k_stfill<float>, dim3((nm + 255) / 256), dim3(256), 0, s, L.metric32.p, (int64_t)nm, 21u, 4, 0, 1.0f);
      hipLaunchKernelGGL(k_stfill<float>, dim3((nb + 255) / 256), dim3(256), 0, s, L.basis32.p, (int64_t)nb, 22u, 1, -1, 0.0f);
    }
    CK(hipDeviceSynchronize());
  }
  const size_t nv = (size_t)L.R * ldb;
  T *x = dalloc<T>(nv), *r = dalloc<T>(nv), *zo = dalloc<T>(nv), *zs = dalloc<T>(nv), *y = dalloc<T>(nv);
  T *ry = dalloc<T>(nv), *rz = dalloc<T>(nv);
  const unsigned g1 = (unsigned)((nv + 255) / 256);
  hipLaunchKernelGGL(k_fill<T>, dim3(g1), dim3(256), 0, s, x, L.R, ldb, W, n1, p, 1u, 1);
  hipLaunchKernelGGL(k_fill<T>, dim3(g1), dim3(256), 0, s, r, L.R, ldb, W, n1, p, 2u, 1);
  hipLaunchKernelGGL(k_fill<T>, dim3(g1), dim3(256), 0, s, zs, L.R, ldb, W, n1, p, 3u, 1);
  CK(hipDeviceSynchronize());
  std::vector<T> ca(ldb, T(1)), cb(ldb, T(1)), c1(ldb), c2(ldb);
  std::mt19937 rng(5);
  std::uniform_real_distribution<double> U(0.2, 0.8);
  for (int c = 0; c < ldb; ++c) {
    if (c < ncols) ca[c] = (T)(1.0 + (c / nsamp) * 0.37);
    c1[c] = (T)U(rng);
    c2[c] = (T)U(rng);
  }
  int nslot = 0;
  for (int t = 0; t < nt; ++t) {
    std::vector<T> d;
    for (int c = t * 64; c < t * 64 + 64; ++c) {
      bool f = false;
      for (T v : d) f = f || v == ca[c];
      if (!f) d.push_back(ca[c]);
    }
    nslot = std::max(nslot, (int)d.size());
  }
  T *dca = dalloc<T>(ldb), *dcb = dalloc<T>(ldb), *dc1 = dalloc<T>(ldb), *dc2 = dalloc<T>(ldb);
  CK(hipMemcpy(dca, ca.data(), ldb * sizeof(T), hipMemcpyHostToDevice));
  CK(hipMemcpy(dcb, cb.data(), ldb * sizeof(T), hipMemcpyHostToDevice));
  CK(hipMemcpy(dc1, c1.data(), ldb * sizeof(T), hipMemcpyHostToDevice));
  CK(hipMemcpy(dc2, c2.data(), ldb * sizeof(T), hipMemcpyHostToDevice));
  const int nslots_part = partial_slots(L, ldb, nt) + 8;
  double *partial = dalloc<double>((size_t)nslots_part * ldb);
  int *counter = dalloc<int>(nt);
  ColState *cs = dalloc<ColState>(ldb);
  CK(hipMemset(cs, 0, ldb * sizeof(ColState)));
  unsigned long long *cmp = dalloc<unsigned long long>(2);
  Scratch sc{partial, counter};
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const double rows = 6.0 * n1 * n1;
  for (const auto &kind : kinds) {
    if (kind == "copy") {
      float tot = 0.f;
      for (int k = 0; k < 4; ++k) {
        CK(hipEventRecord(e0, s));
        hipLaunchKernelGGL(k_neg<T>, dim3(g1), dim3(256), 0, s, x, y, (int64_t)nv);
        CK(hipEventRecord(e1, s));
        CK(hipEventSynchronize(e1));
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (k > 0) tot += ms;
      }
      const double us = tot * 1e3 / 3.0, bytes = 2.0 * sizeof(T) * nv;
      std::printf("copy     %9.1f us  %7.1f GB/s (%.3g B read, %.3g B written)\n", us, bytes / (us * 1e-6) / 1e9,
                  bytes / 2, bytes / 2);
      std::fflush(stdout);
      continue;
    }
    if (kind == "sumfact") {
      // matrix-free sum-factorised apply (all colours and the zero fill), 1 warm-up + 3 timed
      float tot = 0.f;
      for (int k = 0; k < 4; ++k) {
        CK(hipEventRecord(e0, s));
        launch_sumfact_apply<T>(L, x, y, dca, dcb, ldb, nt, nullptr, s);
        CK(hipEventRecord(e1, s));
        CK(hipEventSynchronize(e1));
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        if (k > 0) tot += ms;
      }
      const double us = tot * 1e3 / 3.0;
      const int nb1 = p + 1;
      const double flops = (20.0 * nb1 * nb1 * nb1 + 8.0 * nb1 * nb1) * 6.0 * L.nel * L.nel * ncols;
      const double bytes = 2.0 * sizeof(T) * ncols * rows + 4.0 * L.q * L.q * 6.0 * L.nel * L.nel * sizeof(T);
      std::printf("sumfact  q=%d %9.1f us %8.2f TFLOP/s  %7.1f GB/s (algorithmic: %.3g flop, %.3g B)\n", L.q, us,
                  flops / (us * 1e-6) / 1e12, bytes / (us * 1e-6) / 1e9, flops, bytes);
      std::fflush(stdout);
      continue;
    }
    EpiArgs<T> e;
    int vecs = 2;
    if (kind == "cheb") {
      e.kind = EPI_CHEB;
      e.dflags = 4;
      vecs = 4;
    } else if (kind == "chebdot") {
      e.kind = EPI_CHEB;
      e.dflags = 4;
      e.dot = 1;
      e.op = OP_ALPHA;
      vecs = 4;
    } else if (kind == "store") {
      e.kind = EPI_STORE;
      vecs = 2;
    } else if (kind == "storedot") {
      e.kind = EPI_STORE;
      e.dot = 1;
      e.op = OP_ALPHA;
      vecs = 2;
    } else {
      e.kind = EPI_RESID;
      vecs = 3;
    }
    e.y = y;
    e.zout = zo;
    e.r = r;
    e.dM = ddM;
    e.dS = ddS;
    e.sig = dca;
    e.cf1 = dc1;
    e.cf2 = dc2;
    const double bytes = (double)vecs * sizeof(T) * ncols * rows + 2.0 * SS * sizeof(T) * rows;
    bool have_ref = false;
    for (int algo : algos)
      for (int slotmode = 0; slotmode < (algo == 1 ? 3 : 1); ++slotmode)
        for (auto sh : shapes) {
          if (sh.TY == 4 && (sizeof(T) == 8 || p > 3)) continue;
          if (sh.TY == 4 && algo == 0) continue;
          ApplyTune tu;
          tu.TY = sh.TY;
          tu.TX = sh.TX;
          tu.grp = sh.G;
          tu.algo = algo;
          e.nslot = slotmode == 0 ? nslot : 0;  // 0: pair fallback
          e.rows16 = slotmode == 2 ? 1 : 0;
          if (slotmode == 2 && nsamp % 16 != 0) continue;
          // timing: one warm-up and five timed launches (z_prev restored before each)
          float tot = 0.f;
          for (int k = 0; k < 6; ++k) {
            CK(hipMemcpyAsync(zo, zs, nv * sizeof(T), hipMemcpyDeviceToDevice, s));
            apply_fused<T>(L, stM, stS, x, dca, dcb, e, sc, cs, nullptr, ldb, nt, 0.0, 100, s, tu, e0, e1);
            CK(hipEventSynchronize(e1));
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            if (k > 0) tot += ms;
          }
          const double us = tot * 1e3 / 5.0;
          // correctness against the first configuration run
          CK(hipMemcpyAsync(zo, zs, nv * sizeof(T), hipMemcpyDeviceToDevice, s));
          apply_fused<T>(L, stM, stS, x, dca, dcb, e, sc, cs, nullptr, ldb, nt, 0.0, 100, s, tu);
          CK(hipDeviceSynchronize());
          double erry = 0, errz = 0;
          if (!have_ref) {
            CK(hipMemcpy(ry, y, nv * sizeof(T), hipMemcpyDeviceToDevice));
            CK(hipMemcpy(rz, zo, nv * sizeof(T), hipMemcpyDeviceToDevice));
            have_ref = true;
          } else {
            unsigned long long h[2];
            for (int w = 0; w < 2; ++w) {
              CK(hipMemset(cmp, 0, 2 * sizeof(unsigned long long)));
              hipLaunchKernelGGL(k_cmp<T>, dim3(g1), dim3(256), 0, s, w ? zo : y, w ? rz : ry, L.R, ldb, ncols, W, n1,
                                 p, cmp);
              CK(hipMemcpy(h, cmp, sizeof(h), hipMemcpyDeviceToHost));
              double d, m;
              std::memcpy(&d, &h[0], 8);
              std::memcpy(&m, &h[1], 8);
              (w ? errz : erry) = m > 0 ? d / m : d;
            }
          }
          std::printf("%-8s algo=%d %s TY=%d TX=%-3d G=%-2d %9.1f us %7.1f GB/s (%.1f%%)  rel.err y %.2e z %.2e  nslot=%d\n",
                      kind.c_str(), algo, slotmode == 2 ? "dpp " : slotmode ? "pair" : "comb", sh.TY, sh.TX, sh.G, us, bytes / (us * 1e-6) / 1e9,
                      100.0 * bytes / (us * 1e-6) / 8e12, erry, errz, e.nslot);
          std::fflush(stdout);
        }
  }
  for (T *q : {stM, stS, ddM, ddS, x, r, zo, zs, y, ry, rz, dca, dcb, dc1, dc2}) CK(hipFree(q));
  CK(hipFree(partial));
  CK(hipFree(counter));
  CK(hipFree(cs));
  CK(hipFree(cmp));
}

int main(int argc, char **argv) {
  if (argc < 7) {
    std::fprintf(stderr, "usage: %s p lev nnode nsamp f32|f64 kinds [algos] [TY:TX,...]\n", argv[0]);
    return 2;
  }
  const int p = std::atoi(argv[1]), lev = std::atoi(argv[2]), nnode = std::atoi(argv[3]), nsamp = std::atoi(argv[4]);
  const std::string dt = argv[5];
  std::vector<std::string> kinds;
  {
    std::string k = argv[6], cur;
    for (char c : k + ",") {
      if (c == ',') { if (!cur.empty()) kinds.push_back(cur); cur.clear(); } else cur += c;
    }
  }
  std::vector<int> algos{0, 1};
  if (argc > 7) {
    algos.clear();
    for (char c : std::string(argv[7]))
      if (c >= '0' && c <= '9') algos.push_back(c - '0');
  }
  const int G0 = ApplyTune().grp;
  std::vector<Shape> shapes{{1, 32, G0}, {2, 32, G0}, {1, 64, G0}, {2, 64, G0}, {4, 32, G0}, {4, 64, G0}};
  if (argc > 8) {
    shapes.clear();
    std::string k = std::string(argv[8]) + ",", cur;
    for (char c : k) {
      if (c == ',') {
        int a = 0, b = 0, c = G0;
        if (std::sscanf(cur.c_str(), "%d:%d:%d", &a, &b, &c) >= 2) shapes.push_back({a, b, c < 1 ? 1 : c});
        cur.clear();
      } else cur += c;
    }
  }
  if (dt == "f64") run<double>(p, lev, nnode, nsamp, kinds, algos, shapes);
  else run<float>(p, lev, nnode, nsamp, kinds, algos, shapes);
  return 0;
}
