// Device helpers and the combined-stencil operator kernel (included by k_fused.hip).
#pragma once
#include "gf_internal.h"
#include "k_solve.h"

#include <type_traits>

namespace gf {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// (M_i, S_i) coefficient pair of one stencil tap, read from LDS in one instruction
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

// reduce one double per lane over the 4 wavefronts of the block into partial[slot][col]
__device__ __forceinline__ void block_partial(double acc, double *partial, int64_t slot, int ldb, int col) {
  __shared__ double red[4][CT];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0) partial[slot * ldb + col] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// the same for two doubles per lane, into partial[slot0][col] and partial[slot1][col]
__device__ __forceinline__ void block_partial2(double acc0, double acc1, double *partial, int64_t slot0,
                                               int64_t slot1, int ldb, int col) {
  __shared__ double red2[2][4][CT];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  red2[0][w][lane] = acc0;
  red2[1][w][lane] = acc1;
  __syncthreads();
  if (w == 0) {
    partial[slot0 * ldb + col] = red2[0][0][lane] + red2[0][1][lane] + red2[0][2][lane] + red2[0][3][lane];
    partial[slot1 * ldb + col] = red2[1][0][lane] + red2[1][1][lane] + red2[1][2][lane] + red2[1][3][lane];
  }
}

// ------------------------------------------------------------------ combined-stencil kernel
// The same operator and epilogues as k_apply_fused, organised around two observations.
//  * Every system of a column tile applies ca M + cb S with its own (ca, cb); the tiles of the solver
//    hold few distinct pairs (the samples of one sinc node share the shift).  Each wavefront finds the
//    distinct pairs of its tile once (ballot over the lanes), and per output row stages one combined
//    stencil ca_d M_i + cb_d S_i per distinct pair d in its LDS slot; a lane then needs one LDS read and
//    one multiply-add per tap instead of one read and two multiply-adds.  A tile with more distinct
//    pairs than the slots hold falls back to the separate (M_i, S_i) pairs of k_apply_fused.  The
//    Jacobi diagonal of an interior row is the centre of its combined stencil (interior unknowns have
//    one copy), so the smoothing step reads no diagonal vectors.
//  * Vector memory loads return in order, so a load issued after another cannot complete first.  All
//    loads of a step -- the window's next column, the stencils of the next step's rows and the
//    epilogue's right-hand side and previous iterate -- are issued one step ahead, before the arithmetic
//    of the current step; the waits of a step then cover only loads issued a full step earlier.
//    For degrees up to 3 the step loop is unrolled by the stencil width, so the window rotates by
//    register renaming instead of register moves.
template <typename T>
__device__ __forceinline__ T read_lane(T v, int l);
template <>
__device__ __forceinline__ float read_lane<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ double read_lane<double>(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ unsigned long long bit_pattern(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long bit_pattern(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// How a strip applies ca M + cb S (chosen by the host from what it knows of the column tiles):
//   SM_COMB  one combined stencil per distinct (ca, cb) of the tile in LDS, one broadcast read per tap
//   SM_PAIR  the separate M and S stencils in LDS, two reads and two multiply-adds per tap (any tile)
//   SM_DPP   (ca, cb) is the same within each aligned group of 16 columns: every lane combines 16 taps
//            of the stencils with its own (ca, cb) into one register, and each tap is one multiply-add
//            whose coefficient operand is broadcast within the 16 lanes by the DPP row_newbcast
//            modifier -- no LDS read per tap
enum StencilMode { SM_COMB = 0, SM_PAIR = 1, SM_DPP = 2 };

// acc += (lane J of this lane's 16-lane row of c) * x.  The compiler does not fold its own DPP moves
// into multiply-adds, so the instruction is written out; the first tap of a chunk waits the two
// cycles a DPP source written by the previous vector instruction needs (arithmetic only: no memory
// access in the asm).
template <int J, bool FIRST>
__device__ __forceinline__ void fma_row_bcast(float &acc, float c, float x) {
  if constexpr (FIRST)
    asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc) : "v"(c), "v"(x), "i"(J));
  else
    asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc) : "v"(c), "v"(x), "i"(J));
}
template <int J, bool FIRST>
__device__ __forceinline__ void fma_row_bcast(double &acc, double c, double x) {
  if constexpr (FIRST)
    asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc) : "v"(c), "v"(x), "i"(J));
  else
    asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc) : "v"(c), "v"(x), "i"(J));
}
// value of lane J of this lane's 16-lane row
template <int J>
__device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + J, 0xf, 0xf, true));
}
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xf, 0xf, true);
}

// In DPP mode the taps are summed column by column: the o-th multiply-add of a row's chain takes tap
// (dy, dx) = (o mod S, o / S), tap index dy S + dx.  The window's leftmost column (dx = 0) is then dead
// after the first S multiply-adds of every row, and the next column is loaded into its registers while
// the other columns are summed (no staging registers for it).  The LDS modes sum row by row (tap
// order), which lets the compiler read the coefficients of consecutive taps in wide LDS reads.
template <int S>
constexpr int tap_at(int o) {
  return (o % S) * S + o / S;
}
// whether the o-th multiply-add is the first to read its 16-tap chunk register
template <int S>
constexpr bool chunk_first(int o) {
  for (int k = 0; k < o; ++k)
    if (tap_at<S>(k) / 16 == tap_at<S>(o) / 16) return false;
  return true;
}

// acc[t] += the multiply-adds o in [O, O1) of the NT rows of a step, in DPP mode: tap (dy, dx) takes its
// coefficient from chunk tap / 16, lane tap % 16, and the window column (u + dx) mod U of row t + dy;
// the rows' chains are interleaved (independent multiply-adds back to back)
template <typename T, int S, int U, int NT, int O, int O1, typename Win>
__device__ __forceinline__ void dpp_taps(T (&acc)[NT], const T (&c)[NT][(S * S + 15) / 16], const Win &win, int u) {
  if constexpr (O < O1) {
    constexpr int tap = tap_at<S>(O), dy = tap / S, dx = tap % S;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      fma_row_bcast<tap % 16, chunk_first<S>(O)>(acc[t], c[t][tap / 16], win[t + dy][(U == S) ? (u + dx) % S : dx]);
    dpp_taps<T, S, U, NT, O + 1, O1>(acc, c, win, u);
  }
}

// the stencil sum of row t with coefficients from a stencil in LDS (lc[tap]), in tap order
template <typename T, int S, int U, typename Win>
__device__ __forceinline__ T lds_taps(const T *lc, const Win &win, int t, int u) {
  T acc = 0;
#pragma unroll
  for (int o = 0; o < S * S; ++o) {
    const int dy = o / S, dx = o % S;
    acc = fma(lc[o], win[t + dy][(U == S) ? (u + dx) % S : dx], acc);
  }
  return acc;
}

// Raw buffer accesses: a wavefront-uniform 128-bit descriptor (base address in scalar registers) plus a
// 32-bit per-lane offset and a 32-bit uniform offset.  The per-lane offset of a vector access is the
// lane times the element size, fixed for the whole kernel, so no address arithmetic runs per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base) {
  // word 3 = 0x00020000: 32-bit data format, the setting for raw (untyped) buffer access on this
  // architecture; records = 2^31 - 1 bytes (offsets stay far below, see stencil_offsets_fit)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float buf_ld(float, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ double buf_ld(double, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, 0);
}
typedef unsigned int buf_v2u __attribute__((vector_size(8)));
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(buf_v2u, v), r, vo, so, 0);
}

// slots of combined stencils per wavefront: as many as keep the block's LDS at 32 KiB
template <typename T, int P, int TY>
struct StencilSlots {
  static constexpr int SS = (2 * P + 1) * (2 * P + 1);
  static constexpr int value = (4 * TY * 8 * SS * (int)sizeof(T) <= 32768) ? 8 : 4;
};

// One strip of TY rows x [x0, x1) of one patch for one column tile (lane = system), in stencil mode
// MODE.  Returns the lane's share of the epilogue's inner product.
template <typename T, int P, int TY, int KIND, int DOT, int MODE, typename XT>
__device__ __forceinline__ double stencil_strip(const ApplyGeom &g, const T *__restrict__ stM,
                                                const T *__restrict__ stS, const XT *__restrict__ x,
                                                T *__restrict__ y, T *__restrict__ zout, const T *__restrict__ r,
                                                int m, int iy0, int x0, int x1, int64_t ct0, int lane, T *lds,
                                                const T *sab, int slot, int nd, T a, T b, T a1, T a2, int dflags,
                                                const double *__restrict__ q2, double &acc2) {
  constexpr int S = 2 * P + 1, SS = S * S, WR = TY + 2 * P, NH = (SS + 63) / 64, NCH = (SS + 15) / 16;
  constexpr bool PAIR = MODE != SM_COMB;
  constexpr int U = (P <= 3) ? S : 1;
  constexpr int MAXD = StencilSlots<T, P, TY>::value;
  const int W = g.W, n1 = g.n1;
  const int64_t ldb = g.ldb;
  const int64_t pbase = (int64_t)m * W * W;
  const bool need_zp = (KIND == EPI_CHEB) && (dflags & 4) && !(dflags & 1);
  // Buffer bases (uniform): the window's first padded row iy0 and the strip's first output row, each
  // at column tile ct0; every offset below is relative to them.  Window rows iy0 .. iy0 + TY + 2P - 1
  // are clamped into the padded patch, output rows to the last coefficient row (a clamped row is read
  // but never written).
  const int64_t wrow0 = pbase + (int64_t)iy0 * W;                   // padded row of window row 0, column 0
  const int64_t orow0 = pbase + (int64_t)(iy0 + P) * W + P;         // row of output (iy0, 0)
  const __amdgpu_buffer_rsrc_t bx = buf_rsrc(x + wrow0 * ldb + ct0);
  const __amdgpu_buffer_rsrc_t br = buf_rsrc(r + orow0 * ldb + ct0);
  const __amdgpu_buffer_rsrc_t bz = buf_rsrc(zout + orow0 * ldb + ct0);
  const __amdgpu_buffer_rsrc_t by = buf_rsrc(y + orow0 * ldb + ct0);
  const __amdgpu_buffer_rsrc_t bm = buf_rsrc(stM + orow0 * SS);
  const __amdgpu_buffer_rsrc_t bs = buf_rsrc(stS + orow0 * SS);
  // dot 2: z_out.q2 with q2 in FP64 (offsets checked by stencil_dot2_fits)
  __amdgpu_buffer_rsrc_t bq;
  if constexpr (DOT == 2) bq = buf_rsrc(q2 + orow0 * ldb + ct0);
  constexpr uint32_t E = sizeof(T);
  const uint32_t colb = (uint32_t)ldb * E;                          // bytes from one row to the next
  const uint32_t vo = (uint32_t)lane * E;                           // this lane's offset in a row
  // the window vector may be stored in a narrower type than the arithmetic (XT = float, T = double:
  // the FP32 search direction of the mixed-precision CG); each value is widened once, when loaded
  constexpr uint32_t EX = sizeof(XT);
  const uint32_t colbx = (uint32_t)ldb * EX, vox = (uint32_t)lane * EX;
  auto ldx = [&](uint32_t so) -> T { return (T)buf_ld(XT(), bx, vox, so); };
  uint32_t woff[WR];
#pragma unroll
  for (int k = 0; k < WR; ++k) woff[k] = (uint32_t)((min(iy0 + k, W - 1) - iy0) * W) * colbx;
  uint32_t ooff[TY];
#pragma unroll
  for (int t = 0; t < TY; ++t) ooff[t] = (uint32_t)((min(iy0 + t, n1 - 1) - iy0) * W);  // in rows

  // columns x0 .. x0 + 2P of the window.  Rotating window (U = S): column x0 + c in slot c; in step u the
  // window's column dx sits in slot (u + dx) mod S, and the column of the next step is loaded into the
  // slot of column dx = 0 once that column's multiply-adds are issued.  Shifting window (U = 1): columns
  // x0 .. x0 + 2P - 1 in slots 1 .. S-1, column x0 + 2P in nxt; each step shifts the slots down by one,
  // appends nxt and loads the next column into nxt before its arithmetic.
  T win[WR][S], nxt[WR];
#pragma unroll
  for (int k = 0; k < WR; ++k) {
    if constexpr (U == S) {
#pragma unroll
      for (int c = 0; c < S; ++c) win[k][c] = ldx(woff[k] + (uint32_t)(x0 + c) * colbx);
    } else {
#pragma unroll
      for (int c = 0; c < S - 1; ++c) win[k][c + 1] = ldx(woff[k] + (uint32_t)(x0 + c) * colbx);
      nxt[k] = ldx(woff[k] + (uint32_t)(x0 + 2 * P) * colbx);
    }
  }
  T cmn[TY][NH], csn[TY][NH], rvn[TY], zpn[TY];
  uint32_t vst[NH];  // this lane's stencil tap, in bytes
#pragma unroll
  for (int h = 0; h < NH; ++h) vst[h] = (uint32_t)min(h * 64 + lane, SS - 1) * E;
  auto load_step = [&](int ixn) {
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const uint32_t orr = ooff[t] + (uint32_t)ixn;  // output row relative to orow0
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        cmn[t][h] = buf_ld(T(), bm, vst[h], orr * (uint32_t)(SS * E));
        csn[t][h] = buf_ld(T(), bs, vst[h], orr * (uint32_t)(SS * E));
      }
      if (KIND != EPI_STORE) rvn[t] = buf_ld(T(), br, vo, orr * colb);
      if (need_zp) zpn[t] = buf_ld(T(), bz, vo, orr * colb);
    }
  };
  load_step(x0);

  double acc = 0.0;
  for (int ixb = x0; ixb < x1; ixb += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ix = ixb + u;
      if (ix >= x1) break;
      const int ixn = min(ix + 1, x1 - 1);
      if constexpr (U != S) {
        // shift the window, append the column loaded during the previous step, load the next one
#pragma unroll
        for (int k = 0; k < WR; ++k) {
#pragma unroll
          for (int c = 0; c < S - 1; ++c) win[k][c] = win[k][c + 1];
          win[k][S - 1] = nxt[k];
          nxt[k] = ldx(woff[k] + (uint32_t)(ixn + 2 * P) * colbx);
        }
      }
      // stage this step's stencils (loaded during the previous step; lane l holds tap l of M_i and
      // S_i), then reuse their registers for the next step's loads
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        T *lt = lds + t * MAXD * SS;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int l = h * 64 + lane;
          if (l < SS) {
            if (PAIR) {
              lt[l] = cmn[t][h];
              lt[SS + l] = csn[t][h];
            } else {
              for (int d = 0; d < nd; ++d) lt[d * SS + l] = sab[2 * d] * cmn[t][h] + sab[2 * d + 1] * csn[t][h];
            }
          }
        }
      }
      T rv[TY], zp[TY];
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        rv[t] = rvn[t];
        zp[t] = zpn[t];
      }
      load_step(ixn);
      // dot 2: q2 at this step's output rows, loaded now and first needed in the epilogue (no
      // registers held across steps for it)
      double qv[TY];
      if constexpr (DOT == 2) {
#pragma unroll
        for (int t = 0; t < TY; ++t)
          qv[t] = buf_ld(double(), bq, (uint32_t)lane * 8u, (ooff[t] + (uint32_t)ix) * (uint32_t)ldb * 8u);
      }
      __builtin_amdgcn_wave_barrier();
      // DPP mode: chunk k of row t holds taps 16k .. 16k+15 of this lane's combined stencil in the
      // lanes of every 16-lane row
      T cc[TY][NCH];
      if (MODE == SM_DPP) {
#pragma unroll
        for (int t = 0; t < TY; ++t)
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            const int tap = min(16 * k + (lane & 15), SS - 1);
            cc[t][k] = (16 * k + (lane & 15) < SS) ? a * lds[t * MAXD * SS + tap] + b * lds[t * MAXD * SS + SS + tap]
                                                   : T(0);
          }
      }
      // DPP mode: the stencil sums of all TY rows before the epilogue, column dx = 0 first, then the
      // next step's newest column into that column's slot.  LDS modes: the next column into nxt now,
      // each row's sum in the epilogue (one row's coefficient reads in flight), nxt into the freed
      // slot after it.
      T ac[TY];
      if constexpr (MODE == SM_DPP) {
#pragma unroll
        for (int t = 0; t < TY; ++t) ac[t] = 0;
        if constexpr (U == S) {
          dpp_taps<T, S, U, TY, 0, S>(ac, cc, win, u);
#pragma unroll
          for (int k = 0; k < WR; ++k) win[k][u % S] = ldx(woff[k] + (uint32_t)(ixn + 2 * P) * colbx);
          dpp_taps<T, S, U, TY, S, S * S>(ac, cc, win, u);
        } else {
          dpp_taps<T, S, U, TY, 0, S * S>(ac, cc, win, u);
        }
      } else if constexpr (U == S) {
#pragma unroll
        for (int k = 0; k < WR; ++k) nxt[k] = ldx(woff[k] + (uint32_t)(ixn + 2 * P) * colbx);
      }
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        const int iy = iy0 + t;
        if (iy >= n1) break;
        const T *lt = lds + t * MAXD * SS;
        T Az, D;
        if (MODE == SM_DPP) {
          Az = ac[t];
          D = row_bcast<(P * S + P) % 16>(cc[t][(P * S + P) / 16]);
        } else if (PAIR) {  // slot 0 holds M_i, slot 1 S_i
          const T am = lds_taps<T, S, U>(lt, win, t, u);
          Az = a * am + b * lds_taps<T, S, U>(lt + SS, win, t, u);
          D = a * lt[P * S + P] + b * lt[SS + P * S + P];
        } else {
          Az = lds_taps<T, S, U>(lt + slot * SS, win, t, u);
          D = lt[slot * SS + P * S + P];
        }
        const uint32_t so = (ooff[t] + (uint32_t)ix) * colb;
        const T zc = win[t + P][(U == S) ? (u + P) % S : P];
        const bool shared = (ix == 0) | (ix == n1 - 1) | (iy == 0) | (iy == n1 - 1);
        if (shared) {
          buf_st(Az, by, vo, so);  // patch contribution; the interface kernel completes it
        } else if (KIND == EPI_STORE) {
          buf_st(Az, by, vo, so);
          if (DOT) acc += (double)zc * (double)Az;
        } else if (KIND == EPI_RESID) {
          buf_st(rv[t] - Az, by, vo, so);
        } else {
          const T dp = (dflags & 4) ? ((dflags & 1) ? zc : zc - zp[t]) : T(0);
          // FP32: the hardware reciprocal (1 ulp) instead of the correctly rounded division, which
          // costs some ten vector instructions per row in this loop; D is a positive diagonal
          T jr;
          if constexpr (sizeof(T) == 4)
            jr = (rv[t] - Az) * __builtin_amdgcn_rcpf(D);
          else
            jr = (rv[t] - Az) / D;
          const T dn = a1 * dp + a2 * jr;
          const T zo = zc + dn;
          buf_st(zo, bz, vo, so);
          if (DOT) acc += (double)rv[t] * (double)zo;
          if constexpr (DOT == 2) acc2 += (double)zo * qv[t];
        }
      }
      if constexpr (MODE != SM_DPP && U == S) {
#pragma unroll
        for (int k = 0; k < WR; ++k) win[k][u % S] = nxt[k];
      }
      // the next step's staging overwrites this step's stencils only after these reads (LDS
      // instructions of one wavefront execute in order)
      __builtin_amdgcn_wave_barrier();
    }
  }
  return acc;
}

// waves per SIMD the register allocation of a stencil kernel is held to (0: the compiler's choice)
template <typename T, int P, int TY, int KIND, int MODE>
struct StencilWaves {
  static constexpr int value = (sizeof(T) == 8 && P == 3 && TY == 2 && KIND == EPI_STORE && MODE == SM_DPP) ? 3 : 0;
};

template <typename T, int P, int TY, int KIND, int DOT, int MODE, typename XT = T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StencilWaves<T, P, TY, KIND, MODE>::value)))
void k_stencil(ApplyGeom g, const T *__restrict__ stM, const T *__restrict__ stS,
                                                 const XT *__restrict__ x, const T *__restrict__ ca,
                                                 const T *__restrict__ cb, const T *__restrict__ cf1,
                                                 const T *__restrict__ cf2, T *__restrict__ y, T *__restrict__ zout,
                                                 const T *__restrict__ r, double *__restrict__ partial,
                                                 const int *__restrict__ active, int dflags,
                                                 const double *__restrict__ q2) {
  constexpr int SS = (2 * P + 1) * (2 * P + 1);
  constexpr int MAXD = StencilSlots<T, P, TY>::value;
  __shared__ __attribute__((aligned(16))) T lds_all[4][TY * MAXD * SS];
  __shared__ T sab_all[4][2 * MAXD];
  const int Lb = blockIdx.x;
  const int bl = (Lb & 7) * g.q + (Lb >> 3);
  if (bl >= g.nsb * g.ntiles) return;
  // groups of grp vertically adjacent strip blocks (the last group may be shorter); within a group the
  // blocks of one column tile run back to back (they share halo rows), then those of the next tile
  // (the tiles share the group's stencil rows).  grp = 1: column tile fastest
  int ct, sb;
  {
    const int per = g.grp * g.ntiles, gi = bl / per, rem = bl - gi * per;
    const int gs = min(g.grp, g.nsb - gi * g.grp);
    ct = rem / gs;
    sb = gi * g.grp + (rem - ct * gs);
  }
  if (active && !active[ct]) return;
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  const int col = ct * CT + lane;
  const int strip = sb * 4 + wave;
  double acc = 0.0, acc2 = 0.0;
  if (strip < g.nstrip) {
    const int iyb = strip % g.nyb;
    const int seg = (strip / g.nyb) % g.nseg;
    const int m = strip / (g.nyb * g.nseg);
    const int iy0 = iyb * TY;
    const int x0 = seg * g.TX, x1 = min(x0 + g.TX, g.n1);
    const T a = ca[col], b = cb[col];
    T a1 = 0, a2 = 0;
    if (KIND == EPI_CHEB) {
      if (dflags & 4) a1 = cf1[col];
      a2 = cf2[col];
    }
    T *sab = sab_all[wave];
    int slot = 0, nd = 0;
    if (MODE == SM_COMB) {
      // distinct (a, b) pairs of the tile by bit pattern (every lane matches itself, so the loop ends
      // after at most 64 rounds); the caller guarantees at most MAXD of them
      unsigned long long rem = ~0ull;
      const unsigned long long ka = bit_pattern(a), kb = bit_pattern(b);
      while (rem) {
        const int l = __builtin_ctzll(rem);
        const T al = read_lane(a, l), bl2 = read_lane(b, l);
        const unsigned long long hit = __ballot(ka == bit_pattern(al) && kb == bit_pattern(bl2));
        if (nd < MAXD) {
          if ((hit >> lane) & 1ull) slot = nd;
          if (lane == 0) {
            sab[2 * nd] = al;
            sab[2 * nd + 1] = bl2;
          }
          ++nd;
        }
        rem &= ~hit;
      }
      __builtin_amdgcn_wave_barrier();
    }
    acc = stencil_strip<T, P, TY, KIND, DOT, MODE, XT>(g, stM, stS, x, y, zout, r, m, iy0, x0, x1, (int64_t)ct * CT,
                                                   lane, lds_all[wave], sab, slot, nd, a, b, a1, a2, dflags, q2,
                                                   acc2);
  }
  if constexpr (DOT == 2)
    block_partial2(acc, acc2, partial, sb, (int64_t)g.nslot2 + sb, (int)g.ldb, col);
  else if (DOT)
    block_partial(acc, partial, sb, (int)g.ldb, col);
}

}  // namespace gf
