// Matrix-core versions of the two N-sized products of each round of
// accelerated RPCholesky (Alg. 2, step 3) for gfx950:
//   colgemm:  C = A(:, S_r) - F F(S_r,:)^T   (N x s_r, contraction over k_r)
//   trsm:     G = C L^{-T} = C Linv^T        (N x s_r, contraction over s_r),
//             written into F(:, k_r : k_r + s_r) with FP64 row norms of G.
//
// Both are computed transposed, C^T = Bm * F^T: the N-row operand (F, or C)
// is the MFMA B operand and the small per-round operand Bm (F(S_r,:)^T, or
// Linv) the A operand.  The BF16 modes keep the N-row operands in a
// panel-blocked copy (see blk_offset) in which a lane's contraction values for
// one row are adjacent, so each lane fetches them with 16-byte loads straight
// from HBM into registers, double-buffered one chunk ahead.  The FP64 and FP32
// products, bound by the matrix cores, read F itself (column-major): a load
// then covers 16 rows of four columns, and no second copy of F is kept.  Bm is pre-arranged in
// contraction chunks and staged through LDS once per workgroup, double-
// buffered and shared by the four wavefronts.  Each wavefront owns 16*NB rows
// and all columns of its column group, so F is read from HBM once per round
// (groups of one row panel run back to back on the same XCD and share its L2).
//
// Arithmetic policies:
//   Pol64     v_mfma_f64_16x16x4f64                       (FP64 mode)
//   Pol32     v_mfma_f32_16x16x4f32                       (FP32 mode)
//   PolBF<3>  v_mfma_f32_16x16x32_bf16, hi*hi + hi*lo + lo*hi, both operands
//             split into a BF16 high part and a BF16 remainder; the N-row
//             operands are stored already split (two BF16 planes), so the
//             contraction loop does no conversion at all
//   PolBF<1>  the same with the high parts only
#include "arpc_common.h"
#include "arpc_launch.h"
#include "arpc_mfma.h"

#include <cstdlib>
#include <type_traits>
#include <utility>

namespace arpc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- policies
// T: arithmetic type of the results; S: storage element of the blocked
// N-row operands; SPLANES: storage planes (hi/lo); KC: contraction indices per
// chunk; RAW: contraction values one lane supplies per chunk and plane;
// NB: 16-row tiles per wavefront; CROW/GROW: bytes per column of a staged
// chunk of Bm in LDS (padded) and in global memory; cmap: accumulator layout.
struct Pol64 {
  using T = double;
  using S = double;
  using Acc = d4;
  static constexpr int KC = 16, RAW = 4, NB = 2, SPLANES = 1, PLANES = 1;
  static constexpr int CROW = KC * 8 + 16, GROW = KC * 8;
  // lane l of the accumulator holds column 4i + l/16 of the 16x16 tile
  __device__ static inline int cmap(int l, int i) { return (l >> 4) + 4 * i; }
};
struct Pol32 {
  using T = float;
  using S = float;
  using Acc = f4;
  static constexpr int KC = 16, RAW = 4, NB = 4, SPLANES = 1, PLANES = 1;
  static constexpr int CROW = KC * 4 + 16, GROW = KC * 4;
  __device__ static inline int cmap(int l, int i) { return 4 * (l >> 4) + i; }
};
template <int PASSES>
struct PolBF {
  using T = float;
  using S = __bf16;
  using Acc = f4;
  static constexpr int KC = 32, RAW = 8, NB = 4;
  static constexpr int SPLANES = (PASSES == 3) ? 2 : 1, PLANES = SPLANES;
  static constexpr int CROW = KC * 2 + 16;  // 80 bytes: conflict-free 16-byte reads
  static constexpr int GROW = KC * 2;
  __device__ static inline int cmap(int l, int i) { return 4 * (l >> 4) + i; }
};

// High part = round-to-nearest BF16, low part = BF16 of the remainder.
__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

constexpr int PANEL_WAVES = 4;
template <class Pol>
constexpr int panel_rows() { return PANEL_WAVES * Pol::NB * 16; }

enum { MODE_COLGEMM = 0, MODE_TRSM = 1 };

// Panel-blocked layout of the N-row operands (the internal copy of F and the
// scratch C).  Rows are grouped in panels of PH = 256; inside a panel the
// contraction index runs in chunks of KC; a chunk holds SPLANES planes, and in
// a plane each row stores its KC values contiguously.  One row panel of the
// whole factor is a single contiguous region (PH rows per panel).  In the 16x16x4 products the
// four values a lane supplies over four successive steps are adjacent indices
// (lane group g supplies 4g .. 4g+3); the staged Bm is read the same way.
template <class Pol>
__host__ __device__ inline size_t blk_offset(int64_t row, int64_t k, int64_t nkc, int plane) {
  return (((size_t)((row / PH) * nkc + k / Pol::KC) * Pol::SPLANES + plane) * PH + (size_t)(row % PH)) * Pol::KC +
         (size_t)(k % Pol::KC);
}

// Arguments of one panel product.
struct PanelArgs {
  const void* Bsrc;    // colgemm: F itself (FP64, FP32; column-major, ld N) or its panel-blocked
                       // copy (BF16 modes); trsm: C, panel-blocked
  int64_t nkc_src;     // contraction chunks per panel of Bsrc
  int64_t N;
  const unsigned char* Bm;  // chunked small operand (see chunk_offset)
  int Ctot;            // padded column count of Bm (multiple of 16)
  const double* X;     // points (colgemm epilogue)
  int d;
  const double* Xp;    // accepted points, s x d
  KParams kp;
  void* out_user;      // F, column-major, ld N (trsm only)
  void* out_blk;       // C (colgemm) or the blocked copy of F (trsm; null in FP64 and FP32), panel-blocked
  int64_t nkc_out;     // contraction chunks per panel of out_blk
  double* P;           // partial row norms (trsm), groups x N
  const RoundState* st;
  int npanels;         // row panels of this kernel
  int ngroups;         // column groups
  const void* C0;      // colgemm: kernel columns precomputed by k_dist (T, column-major, ld N), or null
  // colgemm in the FP8 mode with the distances in the epilogue (see k_panel):
  const unsigned char* X8;   // the rounded points as e4m3 codes, N x d bytes
  const float* xn8;          // their squared norms
  const unsigned char* Xp8;  // the accepted points as e4m3 codes, b x d bytes
  const float* ypn;          // their squared norms
  KFast kf;
};

// Byte offset of element (k, c) of the chunked small operand.
template <class Pol>
__host__ __device__ inline size_t chunk_offset(int64_t k, int c, int Ctot, int plane) {
  const int64_t ch = k / Pol::KC, kk = k % Pol::KC;
  const size_t esz = Pol::GROW / Pol::KC;
  return (size_t)ch * Pol::PLANES * Ctot * Pol::GROW + (size_t)plane * Ctot * Pol::GROW +
         (size_t)c * Pol::GROW + kk * esz;
}

// Store one value into the blocked layout (split into BF16 planes if needed).
template <class Pol>
__device__ inline void store_blk(typename Pol::S* __restrict__ base, int64_t row, int64_t k, int64_t nkc,
                                 typename Pol::T v) {
  if constexpr (Pol::SPLANES == 2) {
    __bf16 hi, lo;
    split_bf16((float)v, hi, lo);
    base[blk_offset<Pol>(row, k, nkc, 0)] = hi;
    base[blk_offset<Pol>(row, k, nkc, 1)] = lo;
  } else {
    base[blk_offset<Pol>(row, k, nkc, 0)] = (typename Pol::S)v;
  }
}

// Store 16 bytes' worth of consecutive columns k .. k + 16 / sizeof(S) - 1
// of one row into the blocked layout (k a multiple of that count, so the piece
// lies in one chunk and is 16-byte aligned), split into BF16 planes if needed.
template <class Pol>
__device__ inline void store_piece(typename Pol::S* __restrict__ base, int64_t row, int64_t k, int64_t nkc,
                                   const typename Pol::T* v) {
  using S = typename Pol::S;
  if constexpr (sizeof(S) == 2) {
    bf8 hi, lo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if constexpr (Pol::SPLANES == 2) {
        __bf16 h, l;
        split_bf16((float)v[j], h, l);
        hi[j] = h;
        lo[j] = l;
      } else {
        hi[j] = (__bf16)v[j];
      }
    }
    // non-temporal: nothing in this launch reads them back, and in L2 they
    // would evict the panel of F that the column groups share
    __builtin_nontemporal_store(hi, (bf8*)(base + blk_offset<Pol>(row, k, nkc, 0)));
    if constexpr (Pol::SPLANES == 2) __builtin_nontemporal_store(lo, (bf8*)(base + blk_offset<Pol>(row, k, nkc, 1)));
  } else {
    u4 w;
    __builtin_memcpy(&w, v, 16);
    __builtin_nontemporal_store(w, (u4*)(base + blk_offset<Pol>(row, k, nkc, 0)));
  }
}

// One lane's slice of the N-row operand for one chunk and one 16-row tile.
template <class Pol>
struct Frag;
template <>
struct Frag<Pol64> {
  d4 v;
};
template <>
struct Frag<Pol32> {
  f4 v;
};
template <int PASSES>
struct Frag<PolBF<PASSES>> {
  bf8 v[PolBF<PASSES>::SPLANES];
};

// --------------------------------------------------------- the panel kernel
// Largest dimension for which a row of X is held in registers in the
// update-GEMM epilogue; larger dimensions stream the coordinates from memory.
constexpr int XREG = 16;
// 16-column blocks per epilogue window (per-wavefront LDS tile of 16*NB rows
// x 64 columns).
constexpr int EPI_CB = 4;

template <class Pol, int NCB>
constexpr int panel_lds_bytes() {
  constexpr int stage = 2 * Pol::PLANES * NCB * 16 * Pol::CROW;
  constexpr int epi = PANEL_WAVES * (Pol::NB * 16 + 1) * EPI_CB * 16 * (int)sizeof(typename Pol::T);
  return stage > epi ? stage : epi;
}

// DIST8 (update GEMM of the FP8 mode, d <= 256, d % 16 == 0): the kernel
// columns are formed in the epilogue from the e4m3 codes instead of being read
// from C0.  Each wavefront stages its 64 rows' codes into its own part of the
// LDS (row stride d + 4 bytes, so the sixteen rows a product reads fall in
// distinct banks) and, per column block, forms x.y on the FP8 matrix cores
// (16x16x32, FP32 accumulation, products exact), with the accepted points'
// codes as the A operand: the result lands in the accumulator layout of the
// update GEMM, so C = kappa - F F(S_r,:)^T is formed in the registers.  r^2 =
// |x|^2 + |y|^2 - 2 x.y, with the direct-difference fallback where it cancels
// (as in k_dist).
// Squared distance of two points given as e4m3 codes, d % 16 == 0: x from
// LDS (4-byte aligned), y from global memory (16-byte aligned).  The
// difference of two e4m3 values is exact in FP32 and the squares are summed in
// FP32, so where the expanded form cancels this keeps the relative accuracy
// of direct differences.  It reads the codes the products read, not the FP64
// points, so a lane that takes it waits for 16-byte loads, not d scattered
// 8-byte ones.
__device__ __attribute__((always_inline)) inline float sqdist_e4m3(const unsigned* x, const unsigned char* y, int d) {
  float s = 0.f;
  for (int q = 0; q < d / 16; ++q) {
    const u4 yv = *(const u4*)(y + 16 * q);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int xw = (int)x[4 * q + w], yw = (int)yv[w];
      const float e0 = __builtin_amdgcn_cvt_f32_fp8(xw, 0) - __builtin_amdgcn_cvt_f32_fp8(yw, 0);
      const float e1 = __builtin_amdgcn_cvt_f32_fp8(xw, 1) - __builtin_amdgcn_cvt_f32_fp8(yw, 1);
      const float e2 = __builtin_amdgcn_cvt_f32_fp8(xw, 2) - __builtin_amdgcn_cvt_f32_fp8(yw, 2);
      const float e3 = __builtin_amdgcn_cvt_f32_fp8(xw, 3) - __builtin_amdgcn_cvt_f32_fp8(yw, 3);
      s = fmaf(e0, e0, s);
      s = fmaf(e1, e1, s);
      s = fmaf(e2, e2, s);
      s = fmaf(e3, e3, s);
    }
  }
  return s;
}

template <class Pol, int NCB, int MODE, int PASSES, bool DIST8 = false>
__global__ __launch_bounds__(64 * PANEL_WAVES) void k_panel(PanelArgs a) {
  using T = typename Pol::T;
  using S = typename Pol::S;
  using Acc = typename Pol::Acc;
  const RoundState* st = a.st;
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  if (s == 0) return;
  const int64_t kr = st->k_r;
  // Blocks are dealt round-robin to the 8 XCDs (each with its own L2).  Block
  // b runs on XCD b % 8; the column groups of one row panel get consecutive
  // slots on the same XCD so that the panel of F they share is read from HBM
  // once and from that XCD's L2 afterwards.
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int grp = slot % a.ngroups;
  const int panel = (slot / a.ngroups) * 8 + xcd;
  if (panel >= a.npanels) return;
  const int cb0 = grp * NCB;                        // first 16-column block of this group
  const int ncb_tot = (s + 15) >> 4;
  if (cb0 >= ncb_tot) return;
  const int ncb = (ncb_tot - cb0) < NCB ? (ncb_tot - cb0) : NCB;
  // contraction length; the inverse factor is lower triangular, so the columns
  // of this group need t < 16 * (cb0 + ncb) only.  The blocked operands hold
  // zeros from the contraction length up to the end of its chunk.
  int64_t K;
  if (MODE == MODE_COLGEMM) K = kr;
  else K = (16 * (cb0 + ncb) < s) ? 16 * (cb0 + ncb) : s;
  const int64_t nchunks = (K + Pol::KC - 1) / Pol::KC;

  constexpr int NB = Pol::NB;
  constexpr int WROWS = NB * 16;                     // rows per wavefront
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t N = a.N;
  const int64_t row_w = (int64_t)panel * panel_rows<Pol>() + (int64_t)w * WROWS;

  constexpr int CP = NCB * 16;                       // columns staged per block
  constexpr int STAGE = Pol::PLANES * CP * Pol::CROW; // LDS bytes per chunk
  __shared__ __attribute__((aligned(16))) unsigned char lds[panel_lds_bytes<Pol, NCB>()];

  Acc acc[NB][NCB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[nb][cb] = Acc{0, 0, 0, 0};

  // ---- staging of the small operand: chunk ch -> LDS buffer, via registers;
  // columns past this group's valid ones are zero-filled
  const int cvalid = 16 * ncb;
  constexpr int Q = Pol::GROW / 16;  // 16-byte pieces per column per chunk
  constexpr int PIECES = Pol::PLANES * CP * Q;
  constexpr int PER_T = (PIECES + 64 * PANEL_WAVES - 1) / (64 * PANEL_WAVES);
  u4 sbuf[PER_T];
  auto fetch = [&](int64_t ch) {
#pragma unroll
    for (int r = 0; r < PER_T; ++r) {
      const int o = tid + r * 64 * PANEL_WAVES;
      const int plane = o / (CP * Q), rem = o % (CP * Q), c = rem / Q, q = rem % Q;
      if (o < PIECES)
        sbuf[r] = (c < cvalid) ? *(const u4*)(a.Bm + (size_t)ch * Pol::PLANES * a.Ctot * Pol::GROW +
                                              (size_t)plane * a.Ctot * Pol::GROW +
                                              (size_t)(16 * cb0 + c) * Pol::GROW + q * 16)
                               : u4{0, 0, 0, 0};
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int r = 0; r < PER_T; ++r) {
      const int o = tid + r * 64 * PANEL_WAVES;
      const int plane = o / (CP * Q), rem = o % (CP * Q), c = rem / Q, q = rem % Q;
      if (o < PIECES) *(u4*)(lds + buf * STAGE + plane * CP * Pol::CROW + c * Pol::CROW + q * 16) = sbuf[r];
    }
  };

  // ---- this lane's slice of the N-row operand: rows row_w + 16 nb + l16,
  // contraction indices k0 + RAW g .. k0 + RAW g + RAW - 1 of each plane.
  // Rows past N lie in the allocated padding of the last panel and only feed
  // outputs that are never stored.
  const S* __restrict__ Bsrc = (const S*)a.Bsrc;
  const int64_t myrow = row_w + l16;                 // row of tile 0
  const S* __restrict__ rowbase = Bsrc + (size_t)(myrow / PH) * a.nkc_src * Pol::SPLANES * PH * Pol::KC +
                                  (size_t)(myrow % PH) * Pol::KC + (size_t)(Pol::RAW * g);
  constexpr size_t CHUNK_ELEMS = (size_t)Pol::SPLANES * PH * Pol::KC;
  constexpr size_t PLANE_ELEMS = (size_t)PH * Pol::KC;
  using F = Frag<Pol>;
  auto load = [&](F (&f)[NB], int64_t ch) {
    if constexpr (Pol::KC == 16 && MODE == MODE_COLGEMM) {
      // FP64 and FP32: F itself, column-major (ld N).  Lane (g, l16) takes
      // columns 16 ch + 4 g .. + 3 of its rows: each load covers 16
      // consecutive rows of four columns (four 128-byte runs in FP64).
      // Columns past k_r are zero (the caller's F holds anything there);
      // rows past N read row N - 1 and feed only outputs that are never stored.
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        int64_t r = myrow + 16 * nb;
        if (r >= N) r = N - 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t k = ch * Pol::KC + 4 * g + i;
          const T v = Bsrc[(size_t)(k < K ? k : K - 1) * N + r];
          f[nb].v[i] = k < K ? v : (T)0;
        }
      }
      return;
    }
    const S* p = rowbase + (size_t)ch * CHUNK_ELEMS;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const S* q = p + (size_t)nb * 16 * Pol::KC;   // tiles of one wavefront share a panel
      if constexpr (Pol::KC == 32) {
#pragma unroll
        for (int pl = 0; pl < Pol::SPLANES; ++pl) f[nb].v[pl] = *(const bf8*)(q + pl * PLANE_ELEMS);
      } else {
        f[nb].v = *(const decltype(f[nb].v)*)q;
      }
    }
  };
  auto compute = [&](const F (&f)[NB], const unsigned char* Ls) {
    if constexpr (Pol::KC == 32) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const bf8 ah = *(const bf8*)(Ls + (cb * 16 + l16) * Pol::CROW + g * 16);
        bf8 al;
        if (PASSES == 3) al = *(const bf8*)(Ls + CP * Pol::CROW + (cb * 16 + l16) * Pol::CROW + g * 16);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, f[nb].v[0], acc[nb][cb], 0, 0, 0);
          if constexpr (PASSES == 3) {
            acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, f[nb].v[1], acc[nb][cb], 0, 0, 0);
            acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, f[nb].v[0], acc[nb][cb], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        T aq[4];
        __builtin_memcpy(aq, Ls + (cb * 16 + l16) * Pol::CROW + 4 * g * sizeof(T), 4 * sizeof(T));
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            if constexpr (sizeof(T) == 8)
              acc[nb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[ks], f[nb].v[ks], acc[nb][cb], 0, 0, 0);
            else
              acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[ks], f[nb].v[ks], acc[nb][cb], 0, 0, 0);
          }
      }
    }
  };

  // ---- contraction loop: the N-row operand one chunk ahead in two register
  // buffers taken in turn, the small operand one chunk ahead, LDS buffer =
  // chunk parity; one barrier per chunk.  FP64 and FP32 products run it
  // straight-line: past the last chunk the loads repeat it (clamped index)
  // and the commit fills the LDS buffer no product reads again, so the waits
  // before each commit count exactly the loads issued after the fetch (about
  // 4% faster in FP64).  The BF16 products guard the last chunk's loads instead,
  // which measured faster for them.
  F fr[2][NB];
  if constexpr (Pol::KC == 16) {
    if (nchunks > 0) {
      fetch(0);
      commit(0);
      load(fr[0], 0);
    }
    __syncthreads();
    for (int64_t ch0 = 0; ch0 < nchunks; ch0 += 2) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t ch = ch0 + u;
        if (ch < nchunks) {   // uniform
          const int64_t nx = ch + 1 < nchunks ? ch + 1 : nchunks - 1;
          fetch(nx);
          load(fr[1 - u], nx);
          compute(fr[u], lds + (ch & 1) * STAGE);
          commit((ch + 1) & 1);
          __syncthreads();
        }
      }
    }
  } else {
    // BF16: the N-row operand FD - 1 chunks ahead in FD register buffers
    // taken in turn (three in the one-product mode, whose registers allow
    // it: the epilogue sets the kernel's peak), the small operand one chunk
    // ahead.  Straight-line as in the FP64 and FP32 loop: the loads and the
    // commit are unconditional (clamped chunk index; past the last chunk
    // the commit fills the LDS buffer no product reads again), only the
    // products are guarded, so the waits stay exact and the loads stay in
    // flight across iterations.
    constexpr int FD = PASSES == 1 ? 3 : 2;
    F fq[FD][NB];
    const int64_t last = nchunks > 0 ? nchunks - 1 : 0;
    if (nchunks > 0) {
      fetch(0);
      commit(0);
#pragma unroll
      for (int u = 0; u < FD - 1; ++u) load(fq[u], u < last ? u : last);
    }
    __syncthreads();
    for (int64_t ch0 = 0; ch0 < nchunks; ch0 += FD) {
#pragma unroll
      for (int u = 0; u < FD; ++u) {
        const int64_t ch = ch0 + u;
        fetch(ch + 1 < last ? ch + 1 : last);
        load(fq[(u + FD - 1) % FD], ch + FD - 1 < last ? ch + FD - 1 : last);
        if (ch < nchunks) compute(fq[u], lds + (ch & 1) * STAGE);
        commit((ch + 1) & 1);
        __syncthreads();
      }
    }
  }

  if constexpr (DIST8) {
    // the staging ring is free (the loop ended with a barrier); wavefront w's
    // rows (64 RS <= 16640 bytes) go to the start of its own epilogue window
    // E (the same offset as E below), which only it touches from here on
    const int dd = a.d, RS = dd + 4, parts = dd / 16;
    constexpr size_t EBYTES = (size_t)(WROWS + 1) * EPI_CB * 16 * sizeof(T);
    static_assert(64 * (256 + 4) <= EBYTES, "staged rows fit the epilogue window");
    unsigned* rowsL = (unsigned*)(lds + (size_t)w * EBYTES);
    // 16-byte pieces, eight loads in flight per lane (a loop with one load
    // per iteration would wait out the latency of each)
    for (int q0 = 0; q0 < 64 * parts; q0 += 64 * 8) {
      u4 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int q = q0 + 64 * j + lane;
        const int qc = q < 64 * parts ? q : 64 * parts - 1;
        const int r = qc / parts, pc = qc % parts;
        int64_t rr = row_w + r;
        if (rr >= N) rr = N - 1;
        v[j] = *(const u4*)(a.X8 + (size_t)rr * dd + 16 * pc);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int q = q0 + 64 * j + lane;
        if (q < 64 * parts) {
          const int r = q / parts, pc = q % parts;
          unsigned* dst = rowsL + (r * RS + 16 * pc) / 4;
          dst[0] = v[j][0];
          dst[1] = v[j][1];
          dst[2] = v[j][2];
          dst[3] = v[j][3];
        }
      }
    }
    // zero codes in each row's pad and (d < 256) in the 256 bytes after the
    // last row: the steps below read up to 256 bytes from a row's start in
    // every lane and zero the A operand past d, so what a lane reads past d
    // must be a finite code (a NaN code would survive the zero operand);
    // 64 (d + 4) + 256 <= 16640 bytes for d <= 248
    rowsL[(lane * RS + dd) / 4] = 0u;
    if (dd < 256) rowsL[(64 * RS) / 4 + lane] = 0u;
    float xn[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      int64_t rr = row_w + 16 * nb + l16;
      xn[nb] = a.xn8[rr < N ? rr : N - 1];
    }
    const float frac = 0x1p-6f;
    // The A operand (accepted points' codes) of a column block for all its
    // 32-wide steps (at most 8 at d <= 256) in registers, the next block's
    // loaded while this one's products run.  A lane's 8 dims are all inside
    // d or all past it (d % 16 == 0); past it both operands are zero.
    constexpr int KS = 8;
    auto load_ap = [&](long (&ap)[KS], int cb) __attribute__((always_inline)) {
      const int cl = 16 * (cb0 + cb) + l16;                   // A operand: column of this lane
      const unsigned char* xa = a.Xp8 + (size_t)(cl < s ? cl : s - 1) * dd + 8 * g;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) ap[kk] = (32 * kk + 8 * g < dd) ? *(const long*)(xa + 32 * kk) : 0l;
    };
    constexpr bool APN = NCB <= 5;   // registers for the next block's operand
    // this lane's staged bytes 8 g .. of its rows 16 nb + l16 (a 32-wide step
    // is a constant offset from here)
    const unsigned* rowp[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) rowp[nb] = rowsL + ((16 * nb + l16) * RS + 8 * g) / 4;
    // squared norms of this lane's four columns of a block
    auto load_y = [&](float (&y)[4], int cb) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * (cb0 + cb) + 4 * g + i;
        y[i] = a.ypn[c < s ? c : s - 1];
      }
    };
    long apc[KS], apn[KS];
    float yc[4];
    load_ap(apc, 0);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (cb < ncb) {   // uniform
        // this block's norms, their latency covered by its products
        load_y(yc, cb);
        if (!APN && cb > 0) load_ap(apc, cb);
        if (APN && cb + 1 < ncb) load_ap(apn, cb + 1);
        f4 dp[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) dp[nb] = f4{0.f, 0.f, 0.f, 0.f};
        // all eight steps, straight-line (a guard per step would split the
        // accumulators across blocks); past d the A operand is zero and the
        // B bytes are finite codes, so those products add exactly zero
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const unsigned* src = rowp[nb] + 8 * kk;
            const long bp = (long)((unsigned long)src[0] | ((unsigned long)src[1] << 32));
            dp[nb] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(apc[kk], bp, dp[nb], 0, 0, 0);
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * (cb0 + cb) + 4 * g + i;
          const float y = yc[i];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int64_t rr = row_w + 16 * nb + l16;
            float r2 = xn[nb] + y - 2.f * dp[nb][i];
            if (__builtin_expect(r2 < frac * (xn[nb] + y), 0)) {   // cancellation: direct differences
              // from the codes (the 13-block group, an override, keeps the
              // FP64 points: the code form inlined there spills)
              if constexpr (NCB <= 8)
                r2 = sqdist_e4m3(rowsL + ((16 * nb + l16) * RS) / 4, a.Xp8 + (size_t)(c < s ? c : s - 1) * dd, dd);
              else
                r2 = (float)sqdist(a.X + (rr < N ? rr : N - 1) * dd, a.Xp + (int64_t)(c < s ? c : s - 1) * dd, dd);
            }
            acc[nb][cb][i] = kappa_fast(r2 > 0.f ? r2 : 0.f, a.kf) - acc[nb][cb][i];
          }
        }
        // the next block's operands become the current ones (after their last use)
        if constexpr (APN) {
#pragma unroll
          for (int kk = 0; kk < KS; ++kk) apc[kk] = apn[kk];
        }
      }
    }
  }

  // ------------------------------------------------------------- epilogue
  // Windows of 64 columns:
  //  A. accumulator tiles -> LDS tile E[col][row] of this wavefront;
  //  B. each lane owns a row: kernel value (update GEMM) or row norm and the
  //     column-major store of F (solve), result written back into E;
  //  C. copy of E into the blocked layout, one row (64 consecutive columns)
  //     per wavefront store.  The group that holds the last column also
  //     writes zeros up to the end of that column's chunk.
  constexpr int EROW = WROWS + 1;                    // padded row count of E
  T* E = (T*)lds + w * EROW * EPI_CB * 16;
  constexpr int LPR = 64 / WROWS;                    // lanes per row (1 or 2)
  const int my_row = lane % WROWS, my_part = lane / WROWS;
  const int64_t row = row_w + my_row;
  const bool rok = row < N;
  const int d = a.d;
  S* __restrict__ ob = (S*)a.out_blk;
  T* __restrict__ ou = (T*)a.out_user;
  const int64_t cshift = (MODE == MODE_COLGEMM) ? 0 : kr;   // blocked column of column c
  // Columns written to the blocked layout: this group's columns; the last
  // group writes exactly up to the end of the chunk holding column s-1 (its
  // data columns, then zeros), never past it: beyond lies the next chunk or,
  // after the last chunk, the next row panel.
  const int clo = 16 * cb0;
  const int cend = (16 * (cb0 + ncb) < s) ? 16 * (cb0 + ncb) : s;  // end of this group's data columns
  int chi = 16 * (cb0 + ncb);
  if (cb0 + ncb >= ncb_tot) chi = (int)((cshift + s + Pol::KC - 1) / Pol::KC * Pol::KC - cshift);
  double xr[XREG];
  if (MODE == MODE_COLGEMM && rok && d <= XREG) {
#pragma unroll
    for (int t = 0; t < XREG; ++t) xr[t] = (t < d) ? a.X[row * d + t] : 0.0;
  }
  double g2 = 0.0;
  for (int w0 = clo; w0 < chi; w0 += 16 * EPI_CB) {
    const int e0 = (w0 - clo) >> 4;                  // first column block of the window
    // A
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        if (cb >= e0 && cb < e0 + EPI_CB && cb < ncb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            E[((cb - e0) * 16 + Pol::cmap(lane, i)) * EROW + nb * 16 + l16] = (T)acc[nb][cb][i];
    __syncthreads();
    // valid columns in the window: this group's data columns only (a window
    // can reach past the group into columns another workgroup owns)
    int wv = cend - w0;
    if (wv > 16 * EPI_CB) wv = 16 * EPI_CB;
    // B
    if (rok) {
#pragma unroll 2
      for (int cc = my_part; cc < wv; cc += LPR) {
        const int c = w0 + cc;
        T& v = E[cc * EROW + my_row];
        if (MODE == MODE_COLGEMM && DIST8) {
          // C formed in the registers before the window
        } else if (MODE == MODE_COLGEMM && a.C0) {
          v = (T)((double)((const T*)a.C0)[(int64_t)c * N + row] - (double)v);
        } else if (MODE == MODE_COLGEMM) {
          const double* xp = a.Xp + (int64_t)c * d;
          double r2 = 0.0;
          if (d <= XREG) {
            double r2b = 0.0;
#pragma unroll
            for (int t = 0; t < XREG; t += 2) {
              if (t < d) {
                const double e = xr[t] - xp[t];
                r2 += e * e;
              }
              if (t + 1 < d) {
                const double e = xr[t + 1] - xp[t + 1];
                r2b += e * e;
              }
            }
            r2 += r2b;
          } else {
            r2 = sqdist(a.X + row * d, xp, d);
          }
          double kap;
          if (sizeof(T) == 8) kap = kappa_r2(r2, a.kp);
          else kap = (double)kappa_r2_f32((float)r2, a.kp);
          v = (T)(kap - (double)v);
        } else {
          ou[(kr + c) * N + row] = v;
          g2 += (double)v * (double)v;
        }
      }
    }
    __syncthreads();
    // C: 16-byte pieces on the piece grid of the blocked layout (a lane
    // per piece, several pieces in flight); a piece that the window covers
    // only in part is written element by element, since its other columns
    // belong to another window or workgroup
    int wend = chi - w0;
    if (wend > 16 * EPI_CB) wend = 16 * EPI_CB;
    if (ob) {   // the solve of the FP64 and FP32 modes keeps no blocked copy of F
      constexpr int PE = 16 / (int)sizeof(S);
      const int64_t a0 = cshift + w0;                    // blocked column of window column 0
      const int64_t p0 = a0 / PE * PE;                   // first piece
      const int npc = (int)((a0 + wend - p0 + PE - 1) / PE);
#pragma unroll 4
      for (int q = lane; q < WROWS * npc; q += 64) {
        const int rl = q / npc, pc = q % npc;
        const int64_t rw = row_w + rl;
        if (rw < N) {
          const int c0 = (int)(p0 + (int64_t)pc * PE - a0);   // window column of the piece's first element
          T v[PE];
#pragma unroll
          for (int j = 0; j < PE; ++j) {
            const int cc = c0 + j;
            v[j] = (cc >= 0 && cc < wv) ? E[cc * EROW + rl] : (T)0;
          }
          if (c0 >= 0 && c0 + PE <= wend) {
            store_piece<Pol>(ob, rw, a0 + c0, a.nkc_out, v);
          } else {
#pragma unroll
            for (int j = 0; j < PE; ++j)
              if (c0 + j >= 0 && c0 + j < wend) store_blk<Pol>(ob, rw, a0 + c0 + j, a.nkc_out, v[j]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (MODE == MODE_TRSM) {
    if (LPR == 2) g2 += __shfl_xor(g2, 32, 64);
    if (my_part == 0 && rok) a.P[(int64_t)grp * N + row] = g2;
  }
}

// ------------------------------------------- kernel columns for large d
// C0(row, c) = kappa(|x_row - x_c|^2) for c < s_r, column-major (ld N), on
// the two-kernel path when d > XREG and in the FP8 mode: the distances come
// from |x|^2 + |y|^2 - 2 x.y with x.y on the matrix cores instead of a d-long
// difference loop per entry.  DM selects the contraction: FP64 16x16x4 (FP64
// mode), FP32 16x16x4 (FP32 and BF16 modes), or FP8 e4m3 16x16x32 with FP32
// accumulation (FP8 mode: the points are already rounded to e4m3, so their
// conversion is exact and so are the products and the squares in FP32).
// Where the expansion cancels (r^2 below a fraction of |x|^2 + |y|^2: 2^-10
// in FP64, 2^-6 otherwise) the entry is recomputed by direct differences in
// FP64, so nearby and identical points keep the direct-difference accuracy.
//
// A workgroup owns 256 rows and 16 CT columns.  The dims go in chunks of DC:
// the workgroup stages the chunk of its rows and columns into LDS in the
// operand format with whole-line loads (LPR lanes per row, four FP64 values
// each; the squares are summed into the norms on the way), then wavefront w
// multiplies rows 64 w .. 64 w + 63 (four row tiles) by all column tiles.
// Operand slots: FP8, byte j of lane group g is dim 8 g + j of the chunk;
// 16x16x4, slot j of lane group g in dim group q is dim 16 q + 4 g + j.
// The kernel values leave one 16-column tile at a time: FP32 ones through
// the wavefront's LDS window (store_tile_cols), FP64 ones straight from the
// accumulators, whose layout already covers whole 128-byte lines.
enum { DIST_F64 = 0, DIST_F32 = 1, DIST_F8 = 2 };

// Column-major store of a wavefront's 64 x 16 FP32 tile of C0 (rows
// row0 .. + 63, columns cbase .. + 15) through its LDS window (16 columns of
// 68 floats): lane (g, l16) holds entry (row 16 rt + l16, column 4 g + i) as
// v[rt][i].  Written back as 16-byte runs of one column per lane, a store
// instruction covers 256-byte pieces of four columns, where storing the
// accumulator entries directly covers 64-byte pieces at 4 bytes per lane.
// The window is the wavefront's own, so no barrier is needed: its LDS writes
// and reads run in program order.  vec: N % 4 == 0, so every run is aligned.
__device__ __attribute__((always_inline)) inline void store_tile_cols(float* win, const float (&v)[4][4], int g,
                                                                      int l16, int lane, float* __restrict__ C0,
                                                                      int64_t N, int64_t row0, int cbase, int s,
                                                                      bool vec) {
  constexpr int WS = 68;   // window column stride: 64 rows + one run of padding, runs stay 16-byte aligned
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) win[(4 * g + i) * WS + 16 * rt + l16] = v[rt][i];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = 64 * q + lane;
    const int col = idx >> 4, rr = 4 * (idx & 15);
    const int c = cbase + col;
    const int64_t row = row0 + rr;
    if (c >= s) continue;
    const float* src = win + col * WS + rr;
    float* dst = C0 + (int64_t)c * N + row;
    if (vec && row + 4 <= N) {
      *(float4*)dst = *(const float4*)src;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (row + j < N) dst[j] = src[j];
    }
  }
}

template <int DM>
struct DistCfg {   // FP32
  typedef float T;      // accumulator and norms
  typedef float Op;     // operand in LDS
  static constexpr int CT = 4, DC = 32, RS = 36;   // RS: LDS row stride in Op (32 + 4 of padding)
};
template <>
struct DistCfg<DIST_F8> {
  typedef float T;
  typedef unsigned char Op;
  static constexpr int CT = 4, DC = 32, RS = 32;
};
template <>
struct DistCfg<DIST_F64> {
  typedef double T;
  typedef double Op;
  static constexpr int CT = 2, DC = 16, RS = 18;
};

template <int DM>
__global__ __launch_bounds__(256) void k_dist(const double* __restrict__ X, int d, const double* __restrict__ Xp,
                                              KParams kp, KFast kf, void* __restrict__ C0v, int64_t N,
                                              int ncb, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  typedef DistCfg<DM> Cfg;
  typedef typename Cfg::T T;
  typedef typename Cfg::Op Op;
  typedef T V4 __attribute__((ext_vector_type(4)));
  constexpr int CT = Cfg::CT, DC = Cfg::DC, RS = Cfg::RS, NC = 16 * CT;
  constexpr int LPR = DC / 4, RPP = 256 / LPR;          // staging: lanes per row, rows per pass
  constexpr int NPR = 256 / RPP, NPC = (NC + RPP - 1) / RPP;
  T* __restrict__ C0 = (T*)C0v;
  const int s = st->s_r;
  // tile order: workgroup i runs on XCD i mod 8; each XCD takes a contiguous
  // range of (row block, column block) tiles, column blocks fastest, so the
  // column blocks of a row block share that XCD's L2 for the rows
  // (the grid is 8 * per workgroups, so tile x per + j is workgroup 8 j + x)
  const int64_t ntile = (N + 255) / 256 * ncb, per = (ntile + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= ntile) return;
  const int64_t rb = t / ncb;
  const int c0 = (int)(t % ncb) * NC;
  if (c0 >= s) return;
  __shared__ __attribute__((aligned(16))) Op rowsL[256 * RS];
  __shared__ __attribute__((aligned(16))) Op colsL[NC * RS];
  __shared__ T xnl[256], ynl[NC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int sl = tid % LPR, sr = tid / LPR;             // staging lane: dims 4 sl .. + 3 of row sr (+ RPP p)
  const int64_t r0 = rb * 256;
  const double* sx[NPR];
  const double* sc[NPC];
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    const int64_t row = r0 + RPP * p + sr;
    sx[p] = X + (row < N ? row : N - 1) * d + 4 * sl;
  }
#pragma unroll
  for (int p = 0; p < NPC; ++p) {
    const int c = c0 + RPP * p + sr;
    sc[p] = Xp + (int64_t)(c < s ? c : s - 1) * d + 4 * sl;
  }
  T nx[NPR], ny[NPC];
#pragma unroll
  for (int p = 0; p < NPR; ++p) nx[p] = 0;
#pragma unroll
  for (int p = 0; p < NPC; ++p) ny[p] = 0;
  V4 acc[CT][4];   // [column tile][row tile]
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[ct][q] = V4{0, 0, 0, 0};

  // four values -> operand format at LDS element e of buf; squares into nrm
  auto put = [&](Op* buf, int e, const double (&v)[4], T& nrm) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < 4; ++j) nrm += (T)v[j] * (T)v[j];
    if constexpr (DM == DIST_F8) {
      int pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v[0], (float)v[1], 0, false);
      pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v[2], (float)v[3], pk, true);
      *(int*)(buf + e) = pk;
    } else if constexpr (DM == DIST_F32) {
      *(float4*)(buf + e) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
      *(double2*)(buf + e) = double2{v[0], v[1]};
      *(double2*)(buf + e + 2) = double2{v[2], v[3]};
    }
  };
  // one chunk of dims k0 .. k0 + DC - 1; only the last (ragged) chunk guards
  auto chunk = [&](int k0, auto ragged) __attribute__((always_inline)) {
    constexpr bool RG = decltype(ragged)::value;
    double vr[NPR][4], vc[NPC][4];
#pragma unroll
    for (int p = 0; p < NPR; ++p)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (RG) vr[p][j] = k0 + 4 * sl + j < d ? sx[p][k0 + j] : 0.0;
        else vr[p][j] = sx[p][k0 + j];
      }
#pragma unroll
    for (int p = 0; p < NPC; ++p)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (RG) vc[p][j] = k0 + 4 * sl + j < d ? sc[p][k0 + j] : 0.0;
        else vc[p][j] = sc[p][k0 + j];
      }
    __syncthreads();   // the previous chunk's operands are consumed
#pragma unroll
    for (int p = 0; p < NPR; ++p) put(rowsL, (RPP * p + sr) * RS + 4 * sl, vr[p], nx[p]);
#pragma unroll
    for (int p = 0; p < NPC; ++p)
      if (RPP * p + sr < NC) put(colsL, (RPP * p + sr) * RS + 4 * sl, vc[p], ny[p]);
    __syncthreads();
    if constexpr (DM == DIST_F8) {
      long ap[CT], bp[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) bp[q] = *(const long*)(rowsL + (64 * w + 16 * q + l16) * RS + 8 * g);
#pragma unroll
      for (int q = 0; q < CT; ++q) ap[q] = *(const long*)(colsL + (16 * q + l16) * RS + 8 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
          acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ap[ct], bp[rt], acc[ct][rt], 0, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < DC / 16; ++q) {
        Op av[CT][4], bv[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[rt][j] = rowsL[(64 * w + 16 * rt + l16) * RS + 16 * q + 4 * g + j];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int j = 0; j < 4; ++j) av[ct][j] = colsL[(16 * ct + l16) * RS + 16 * q + 4 * g + j];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              if constexpr (DM == DIST_F64)
                acc[ct][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ct][j], bv[rt][j], acc[ct][rt], 0, 0, 0);
              else
                acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ct][j], bv[rt][j], acc[ct][rt], 0, 0, 0);
            }
      }
    }
  };
  const int dfull = d - d % DC;
  for (int k0 = 0; k0 < dfull; k0 += DC) chunk(k0, std::false_type{});
  if (dfull < d) chunk(dfull, std::true_type{});
  // norms: the LPR staging lanes of a row hold its partial sums
#pragma unroll
  for (int m = 1; m < LPR; m <<= 1) {
#pragma unroll
    for (int p = 0; p < NPR; ++p) nx[p] += __shfl_xor(nx[p], m, 64);
#pragma unroll
    for (int p = 0; p < NPC; ++p) ny[p] += __shfl_xor(ny[p], m, 64);
  }
  if (sl == 0) {
#pragma unroll
    for (int p = 0; p < NPR; ++p) xnl[RPP * p + sr] = nx[p];
#pragma unroll
    for (int p = 0; p < NPC; ++p)
      if (RPP * p + sr < NC) ynl[RPP * p + sr] = ny[p];
  }
  __syncthreads();   // also: every wavefront is done with rowsL, which holds the store windows
  const T frac = DM == DIST_F64 ? (T)0x1p-10 : (T)0x1p-6;
  // FP32 results go through a store window (FP32 mode: overlaying rowsL);
  // the FP64 accumulator layout already stores whole 128-byte lines, and the
  // window pass measured slower there
  constexpr int WIN = 4 * 16 * 68 * 4;
  static_assert(DM == DIST_F64 || WIN <= (int)sizeof(rowsL) || DM == DIST_F8, "store windows overlay rowsL");
  __shared__ __attribute__((aligned(16))) unsigned char winL[DM == DIST_F8 ? WIN : 16];
  T* win = (DM == DIST_F8 ? (T*)winL : (T*)rowsL) + w * 16 * 68;
  const bool vec = N % 4 == 0;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    T v[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int rl = 64 * w + 16 * rt + l16;
      const int64_t row = r0 + rl;
      const T xn = xnl[rl];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // accumulator entry i of lane (g, l16): column 16 ct + m, row l16 of the tile
        const int m = DM == DIST_F64 ? g + 4 * i : 4 * g + i;
        const int c = c0 + 16 * ct + m;
        const T y = ynl[16 * ct + m];
        T r2 = xn + y - 2 * acc[ct][rt][i];
        if (__builtin_expect(r2 < frac * (xn + y), 0))   // cancellation: direct differences
          r2 = (T)sqdist(X + (row < N ? row : N - 1) * d, Xp + (int64_t)(c < s ? c : s - 1) * d, d);
        if constexpr (DM == DIST_F64) v[rt][i] = kappa_r2(r2, kp);
        else v[rt][i] = kappa_fast(r2 > 0.f ? r2 : 0.f, kf);
      }
    }
    if constexpr (DM == DIST_F64) {
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = c0 + 16 * ct + g + 4 * i;
          const int64_t row = r0 + 64 * w + 16 * rt + l16;
          if (c < s && row < N) C0[(int64_t)c * N + row] = v[rt][i];
        }
    } else {
      store_tile_cols(win, v, g, l16, lane, C0, N, r0 + 64 * w, c0 + 16 * ct, s, vec);
    }
  }
}

// The FP8 mode's packed points: one wavefront per row, four dims per lane
// per step (the values are on the e4m3 grid, so the conversion is exact);
// the squared norm is summed in FP32 from the same values.
__global__ __launch_bounds__(256) void k_pack_e4m3(const double* __restrict__ Xq, int64_t N, int d,
                                                   unsigned* __restrict__ X8, float* __restrict__ xn) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const int dw = d / 4;
  const double* x = Xq + row * d;
  float s = 0.f;
  for (int q = lane; q < dw; q += 64) {
    const double v0 = x[4 * q], v1 = x[4 * q + 1], v2 = x[4 * q + 2], v3 = x[4 * q + 3];
    int pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v0, (float)v1, 0, false);
    pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v2, (float)v3, pk, true);
    X8[row * dw + q] = (unsigned)pk;
    s += (float)v0 * (float)v0 + (float)v1 * (float)v1 + (float)v2 * (float)v2 + (float)v3 * (float)v3;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) xn[row] = s;
}

// k_dist for the FP8 mode when d % 4 == 0: the rows are staged from the
// packed e4m3 codes (4 bytes per lane per pass instead of 32, prefetched one
// chunk ahead while the current chunk's products run) with their norms from
// the packed norms; the pivot columns are staged from their FP64 copy as in
// k_dist.  Tile order, operand slots and the epilogue are those of k_dist.
__global__ __launch_bounds__(256) void k_dist_f8b(const double* __restrict__ X, int d,
                                                  const unsigned* __restrict__ X8, const float* __restrict__ xn8,
                                                  const double* __restrict__ Xp, KFast kf, float* __restrict__ C0,
                                                  int64_t N, int ncb, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  constexpr int CT = 4, DC = 32, NC = 16 * CT, LPR = DC / 4, RPP = 256 / LPR, NPR = 256 / RPP;
  constexpr int NPC = (NC + RPP - 1) / RPP;
  typedef float V4 __attribute__((ext_vector_type(4)));
  const int s = st->s_r;
  const int64_t ntile = (N + 255) / 256 * ncb, per = (ntile + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= ntile) return;
  const int64_t rb = t / ncb;
  const int c0 = (int)(t % ncb) * NC;
  if (c0 >= s) return;
  __shared__ __attribute__((aligned(16))) unsigned rowsL[256 * DC / 4];
  __shared__ __attribute__((aligned(16))) unsigned char colsL[NC * DC];
  __shared__ float xnl[256], ynl[NC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int sl = tid % LPR, sr = tid / LPR;
  const int64_t r0 = rb * 256;
  const int dw = d / 4;
  {
    const int64_t row = r0 + tid;
    xnl[tid] = xn8[row < N ? row : N - 1];
  }
  const unsigned* sx[NPR];
  const double* sc[NPC];
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    const int64_t row = r0 + RPP * p + sr;
    sx[p] = X8 + (row < N ? row : N - 1) * dw + sl;
  }
#pragma unroll
  for (int p = 0; p < NPC; ++p) {
    const int c = c0 + RPP * p + sr;
    sc[p] = Xp + (int64_t)(c < s ? c : s - 1) * d + 4 * sl;
  }
  float ny[NPC];
#pragma unroll
  for (int p = 0; p < NPC; ++p) ny[p] = 0.f;
  V4 acc[CT][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[ct][q] = V4{0, 0, 0, 0};
  unsigned vr[NPR];
  double vc[NPC][4];
  auto load = [&](int k0) __attribute__((always_inline)) {
    const bool in = k0 + 4 * sl < d;   // whole 4-dim groups (d % 4 == 0)
#pragma unroll
    for (int p = 0; p < NPR; ++p) vr[p] = in ? sx[p][k0 / 4] : 0u;
#pragma unroll
    for (int p = 0; p < NPC; ++p)
#pragma unroll
      for (int j = 0; j < 4; ++j) vc[p][j] = in ? sc[p][k0 + j] : 0.0;
  };
  load(0);
  for (int k0 = 0; k0 < d; k0 += DC) {
    __syncthreads();   // the previous chunk's operands are consumed
#pragma unroll
    for (int p = 0; p < NPR; ++p) rowsL[(RPP * p + sr) * (DC / 4) + sl] = vr[p];
#pragma unroll
    for (int p = 0; p < NPC; ++p)
      if (RPP * p + sr < NC) {
#pragma unroll
        for (int j = 0; j < 4; ++j) ny[p] += (float)vc[p][j] * (float)vc[p][j];
        int pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)vc[p][0], (float)vc[p][1], 0, false);
        pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)vc[p][2], (float)vc[p][3], pk, true);
        *(int*)(colsL + (RPP * p + sr) * DC + 4 * sl) = pk;
      }
    __syncthreads();
    if (k0 + DC < d) load(k0 + DC);   // the next chunk, in flight during the products
    long ap[CT], bp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      bp[q] = *(const long*)((const unsigned char*)rowsL + (64 * w + 16 * q + l16) * DC + 8 * g);
#pragma unroll
    for (int q = 0; q < CT; ++q) ap[q] = *(const long*)(colsL + (16 * q + l16) * DC + 8 * g);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ap[ct], bp[rt], acc[ct][rt], 0, 0, 0);
  }
#pragma unroll
  for (int m = 1; m < LPR; m <<= 1)
#pragma unroll
    for (int p = 0; p < NPC; ++p) ny[p] += __shfl_xor(ny[p], m, 64);
  if (sl == 0)
#pragma unroll
    for (int p = 0; p < NPC; ++p)
      if (RPP * p + sr < NC) ynl[RPP * p + sr] = ny[p];
  __syncthreads();
  const float frac = 0x1p-6f;
  __shared__ __attribute__((aligned(16))) float winL[4 * 16 * 68];   // per-wavefront store windows
  float* win = winL + w * 16 * 68;
  const bool vec = N % 4 == 0;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    float v[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int rl = 64 * w + 16 * rt + l16;
      const int64_t row = r0 + rl;
      const float xn = xnl[rl];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 4 * g + i;
        const int c = c0 + 16 * ct + m;
        const float y = ynl[16 * ct + m];
        float r2 = xn + y - 2 * acc[ct][rt][i];
        if (__builtin_expect(r2 < frac * (xn + y), 0))   // cancellation: direct differences
          r2 = (float)sqdist(X + (row < N ? row : N - 1) * d, Xp + (int64_t)(c < s ? c : s - 1) * d, d);
        v[rt][i] = kappa_fast(r2 > 0.f ? r2 : 0.f, kf);
      }
    }
    store_tile_cols(win, v, g, l16, lane, C0, N, r0 + 64 * w, c0 + 16 * ct, s, vec);
  }
}

void launch_pack_e4m3(hipStream_t s, const double* Xq, int64_t N, int d, unsigned* X8, float* xn) {
  hipLaunchKernelGGL(k_pack_e4m3, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, Xq, N, d, X8, xn);
}

// ------------------------------------------ small operands in chunk layout
// Bm(k, c) = F(S_r(c), k) for the update GEMM (zero outside k < k_r, c < s_r).
template <class Pol, int PASSES>
__global__ __launch_bounds__(256) void k_prep_bm(const double* __restrict__ Fs, int64_t ldf,
                                                 const int32_t* __restrict__ acc, int Ctot,
                                                 unsigned char* __restrict__ Bm, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int64_t K = st->k_r;
  const int64_t Kpad = (K + Pol::KC - 1) / Pol::KC * Pol::KC;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = e / Ctot;
  const int c = (int)(e % Ctot);
  if (k >= Kpad) return;
  const double v = (k < K && c < s) ? Fs[(int64_t)acc[c] * ldf + k] : 0.0;
  if constexpr (Pol::KC == 32) {
    __bf16 hi, lo;
    split_bf16((float)v, hi, lo);
    *(__bf16*)(Bm + chunk_offset<Pol>(k, c, Ctot, 0)) = hi;
    if (PASSES == 3) *(__bf16*)(Bm + chunk_offset<Pol>(k, c, Ctot, 1)) = lo;
  } else {
    *(typename Pol::T*)(Bm + chunk_offset<Pol>(k, c, Ctot, 0)) = (typename Pol::T)v;
  }
}

// The same from the FP32 copy of the rows (F stored in FP32; the values, and
// so Bm, are the same): a thread takes eight consecutive k of one column, two
// aligned 16-byte loads from one row of the copy and one 16-byte store per
// BF16 plane (32 bytes for FP32), where the form above reads one element of a
// different row per lane.
template <class Pol, int PASSES>
__global__ __launch_bounds__(256) void k_prep_bm32(const float* __restrict__ Fs32, int64_t ld32, int64_t nk8,
                                                   const int32_t* __restrict__ acc, int Ctot,
                                                   unsigned char* __restrict__ Bm, const RoundState* st) {
  static_assert(Pol::KC % 8 == 0, "a thread's eight k stay in one chunk");
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int64_t K = st->k_r;
  const int64_t Kpad = (K + Pol::KC - 1) / Pol::KC * Pol::KC;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c64 = e / nk8, k0 = 8 * (e % nk8);
  if (c64 >= Ctot || k0 >= Kpad) return;
  const int c = (int)c64;
  float v[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = 0.0f;
  if (c < s && k0 < K) {
    // the row starts 16-byte aligned and k0 is a multiple of 8
    const float* src = Fs32 + (int64_t)acc[c] * ld32 + k0;
    if (k0 + 8 <= K) {
      const float4 a = *reinterpret_cast<const float4*>(src);
      const float4 b = *reinterpret_cast<const float4*>(src + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (k0 + t < K) v[t] = src[t];
    }
  }
  if constexpr (Pol::KC == 32) {
    __bf16 hi[8], lo[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) split_bf16(v[t], hi[t], lo[t]);
    uint4 w;
    __builtin_memcpy(&w, hi, sizeof(w));
    *(uint4*)(Bm + chunk_offset<Pol>(k0, c, Ctot, 0)) = w;
    if (PASSES == 3) {
      __builtin_memcpy(&w, lo, sizeof(w));
      *(uint4*)(Bm + chunk_offset<Pol>(k0, c, Ctot, 1)) = w;
    }
  } else {
    static_assert(sizeof(typename Pol::T) == sizeof(float), "FP32 elements");
    float4* dst = (float4*)(Bm + chunk_offset<Pol>(k0, c, Ctot, 0));
    dst[0] = make_float4(v[0], v[1], v[2], v[3]);
    dst[1] = make_float4(v[4], v[5], v[6], v[7]);
  }
}

// Inverse of the s x s lower factor L (read from H through the accepted
// indices): workgroup c (four wavefronts) computes column c by forward
// substitution and stores Linv(i, c) as element (k = c, column i) of the
// chunked operand of the triangular-solve product.  Workgroups c >= s write
// the zero padding.  b <= 512: by blocks, operands one block ahead (the tiled
// rejection kernel has left the blocks' inverses in H); else column by column.
template <class Pol, int PASSES>
__global__ __launch_bounds__(256) void k_trinv_bm(LFactor L, int Ctot, unsigned char* __restrict__ Bm,
                                                  const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double x[BMAX];
  __shared__ double xp[REJECT_TILED_BMAX];   // proposal-indexed column (block solve)
  __shared__ double ys[128];
  if (L.b <= REJECT_TILED_BMAX) {
    if (c < s) {   // uniform
      linv_blocks_ahead<4>(L.H, L.acc, L.b, s, c, tid, xp, ys);
      for (int i = tid; i < s; i += 256) x[i] = xp[L.acc[i]];
    }
  } else if (s <= 256) {
    if (w == 0) {
      double r[4];
      linv_column(L, s, c, lane, r);
#pragma unroll
      for (int m = 0; m < 4; ++m) x[lane + 64 * m] = r[m];
    }
  } else if (s <= 512) {
    if (w == 0) {
      double r[8];
      linv_column(L, s, c, lane, r);
#pragma unroll
      for (int m = 0; m < 8; ++m) x[lane + 64 * m] = r[m];
    }
  } else if (c < s) {   // uniform
    for (int i = tid; i < s; i += 256) x[i] = 0.0;
    __syncthreads();
    if (tid == 0) x[c] = 1.0 / L.at(c, c);
    __syncthreads();
    for (int i = c + 1; i < s; ++i) {
      if (w == 0) {
        double p = 0.0;
        for (int t = c + lane; t < i; t += 64) p += L.at(i, t) * x[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
        if (lane == 0) x[i] = -p / L.at(i, i);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int i = tid; i < Ctot; i += 256) {
    const double v = (c < s && i >= c && i < s) ? x[i] : 0.0;
    if constexpr (Pol::KC == 32) {
      __bf16 hi, lo;
      split_bf16((float)v, hi, lo);
      *(__bf16*)(Bm + chunk_offset<Pol>(c, i, Ctot, 0)) = hi;
      if (PASSES == 3) *(__bf16*)(Bm + chunk_offset<Pol>(c, i, Ctot, 1)) = lo;
    } else {
      *(typename Pol::T*)(Bm + chunk_offset<Pol>(c, i, Ctot, 0)) = (typename Pol::T)v;
    }
  }
}

// ------------------------------------------------------------------ launchers
template <class Pol, int PASSES, int NCB>
static void launch_panel(hipStream_t s, const MfmaRound& r, const RoundState* st, int which) {
  const int ncb_tot = r.Ctot / 16;
  const int npanels = (int)((r.N + panel_rows<Pol>() - 1) / panel_rows<Pol>());
  const int ngroups = (ncb_tot + NCB - 1) / NCB;
  const unsigned nblocks = (unsigned)((npanels + 7) / 8) * 8u * (unsigned)ngroups;
  const int64_t nkcF = (r.kmax + Pol::KC - 1) / Pol::KC, nkcC = (r.b + Pol::KC - 1) / Pol::KC;
  if (which == 0) {
    // FP64 and FP32 contract over F itself (column-major), the BF16 modes over its blocked copy
    PanelArgs a1{Pol::KC == 16 ? r.F : r.Fb, nkcF, r.N, r.Bm1, r.Ctot, r.X, r.d, r.Xp, r.kp, nullptr, r.C, nkcC, nullptr, st,
                 npanels, ngroups, r.C0, (const unsigned char*)r.X8, r.xn8, r.Xp8, r.ypn, kfast_of(r.kp)};
    if constexpr (std::is_same<Pol, PolBF<1>>::value) {
      if (r.Xp8) {
        hipLaunchKernelGGL((k_panel<Pol, NCB, MODE_COLGEMM, PASSES, true>), dim3(nblocks), dim3(64 * PANEL_WAVES), 0,
                           s, a1);
        return;
      }
    }
    hipLaunchKernelGGL((k_panel<Pol, NCB, MODE_COLGEMM, PASSES>), dim3(nblocks), dim3(64 * PANEL_WAVES), 0, s, a1);
  } else {
    PanelArgs a2{r.C, nkcC, r.N, r.Bm2, r.Ctot, nullptr, 0, nullptr, r.kp, r.F, r.Fb, nkcF, r.P, st,
                 npanels, ngroups, nullptr, nullptr, nullptr, nullptr, nullptr, KFast{}};
    hipLaunchKernelGGL((k_panel<Pol, NCB, MODE_TRSM, PASSES>), dim3(nblocks), dim3(64 * PANEL_WAVES), 0, s, a2);
  }
}

// Column blocks per workgroup (the accumulators of one wavefront are NB x NCB
// tiles).  Groups that keep two wavefronts on each SIMD (one hides the other's
// HBM latency) are four blocks wide, or five where that takes fewer groups:
// every group reads the whole panel of its left operand.  Five blocks fit
// the register budget except in the three-pass BF16 product; in the solve
// they paid off only in FP64 (the FP32 and BF16 solves carry less per byte).
// Wider groups (7, 8, 13 blocks) read F fewer times but run one wavefront per
// SIMD, which costs more than the extra L2 reads.  ARPC_NCB=4|5|7|8|13
// overrides the choice for both products.  `prec` is the product's precision
// (0 FP64, 1 FP32, 2 BF16x3, 3 BF16), `which` 0 the column product, 1 the solve.
inline int ncb_for(int prec, int which, int ncb_tot) {
  static int forced = -1;
  if (forced < 0) {
    const char* e = getenv("ARPC_NCB");
    forced = e ? atoi(e) : 0;
  }
  if (forced == 4 || forced == 5 || forced == 7 || forced == 8 || forced == 13) return forced;
  const bool five = which == 0 ? prec != 2 : prec == 0;
  return five && (ncb_tot + 4) / 5 < (ncb_tot + 3) / 4 ? 5 : 4;
}

template <class Pol, int PASSES>
static void dispatch(hipStream_t s, const MfmaRound& r, const RoundState* st, int prec, int which) {
  switch (ncb_for(prec, which, r.Ctot / 16)) {
    case 4: launch_panel<Pol, PASSES, 4>(s, r, st, which); break;
    case 5: launch_panel<Pol, PASSES, 5>(s, r, st, which); break;
    case 7: launch_panel<Pol, PASSES, 7>(s, r, st, which); break;
    case 8: launch_panel<Pol, PASSES, 8>(s, r, st, which); break;
    default: launch_panel<Pol, PASSES, 13>(s, r, st, which); break;
  }
}

template <class Pol, int PASSES>
static void prep_impl(hipStream_t s, const MfmaRound& r, const RoundState* st) {
  const int64_t kpad = (r.kmax + Pol::KC - 1) / Pol::KC * Pol::KC;
  bool done = false;
  if constexpr (std::is_same<typename Pol::T, float>::value) {
    if (r.Fs32) {
      const int64_t nk8 = kpad / 8, n = nk8 * r.Ctot;
      hipLaunchKernelGGL((k_prep_bm32<Pol, PASSES>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r.Fs32,
                         fs32_ld(r.ldf), nk8, r.acc, r.Ctot, r.Bm1, st);
      done = true;
    }
  }
  if (!done) {
    const int64_t n = kpad * r.Ctot;
    hipLaunchKernelGGL((k_prep_bm<Pol, PASSES>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, r.Fs, r.ldf,
                       r.acc, r.Ctot, r.Bm1, st);
  }
  const int nblk = (r.b + Pol::KC - 1) / Pol::KC * Pol::KC;
  hipLaunchKernelGGL((k_trinv_bm<Pol, PASSES>), dim3(nblk), dim3(256), 0, s, LFactor{r.H, r.acc, r.b}, r.Ctot, r.Bm2,
                     st);
}

size_t mfma_operand_bytes(int prec, int64_t kmax, int b) {
  const int Ctot = (b + 15) / 16 * 16;
  auto bytes = [&](int KC, int planes, int grow) {
    const int64_t k1 = (kmax + KC - 1) / KC, k2 = (b + KC - 1) / KC;
    return std::pair<size_t, size_t>((size_t)k1 * planes * Ctot * grow, (size_t)k2 * planes * Ctot * grow);
  };
  std::pair<size_t, size_t> p;
  switch (prec) {
    case 0: p = bytes(16, 1, 128); break;
    case 1: p = bytes(16, 1, 64); break;
    case 2: p = bytes(32, 2, 64); break;
    default: p = bytes(32, 1, 64); break;
  }
  return p.first > p.second ? p.first : p.second;
}

int mfma_part_cols(int prec, int b) {
  // the solve writes one partial sum of squares per column group
  return 16 * ncb_for(prec, 1, (b + 15) / 16);
}

size_t mfma_blocked_bytes(int prec, int64_t N, int64_t cols) {
  const int KC = prec <= 1 ? 16 : 32;
  // bytes per element: FP64 8, FP32 4, BF16 hi+lo planes 4, BF16 hi plane 2
  const size_t esz = prec == 0 ? 8 : (prec == 3 ? 2 : 4);
  const int64_t rows = (N + PH - 1) / PH * PH;
  return (size_t)rows * (size_t)((cols + KC - 1) / KC * KC) * esz;
}

void launch_mfma_prep(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st) {
  switch (prec) {
    case 0: prep_impl<Pol64, 1>(s, r, st); break;
    case 1: prep_impl<Pol32, 1>(s, r, st); break;
    case 2: prep_impl<PolBF<3>, 3>(s, r, st); break;
    default: prep_impl<PolBF<1>, 1>(s, r, st); break;
  }
}

bool mfma_dist_contraction(int d) { return d > XREG; }

bool mfma_dist_in_epilogue(int d) { return d <= 256 && d % 16 == 0; }

void launch_dist(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st) {
  const int64_t nrb = (r.N + 255) / 256;
  const KFast kf = kfast_of(r.kp);
  const int ncb = prec == 0 ? (r.b + 31) / 32 : (r.b + 63) / 64;
  const dim3 grid((unsigned)((nrb * ncb + 7) / 8 * 8));   // every XCD range complete (see k_dist)
  if (prec == 0)
    hipLaunchKernelGGL(k_dist<DIST_F64>, grid, dim3(256), 0, s, r.X, r.d, r.Xp, r.kp, kf, r.C0, r.N, ncb, st);
  else if (prec == 4 && r.X8)
    hipLaunchKernelGGL(k_dist_f8b, grid, dim3(256), 0, s, r.X, r.d, r.X8, r.xn8, r.Xp, kf, (float*)r.C0, r.N, ncb,
                       st);
  else if (prec == 4)
    hipLaunchKernelGGL(k_dist<DIST_F8>, grid, dim3(256), 0, s, r.X, r.d, r.Xp, r.kp, kf, r.C0, r.N, ncb, st);
  else
    hipLaunchKernelGGL(k_dist<DIST_F32>, grid, dim3(256), 0, s, r.X, r.d, r.Xp, r.kp, kf, r.C0, r.N, ncb, st);
}

void launch_mfma_colgemm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st) {
  switch (prec) {
    case 0: dispatch<Pol64, 1>(s, r, st, 0, 0); break;
    case 1: dispatch<Pol32, 1>(s, r, st, 1, 0); break;
    case 2: dispatch<PolBF<3>, 3>(s, r, st, 2, 0); break;
    default: dispatch<PolBF<1>, 1>(s, r, st, 3, 0); break;
  }
}

void launch_mfma_trsm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st) {
  switch (prec) {
    case 0: dispatch<Pol64, 1>(s, r, st, 0, 1); break;
    case 1: dispatch<Pol32, 1>(s, r, st, 1, 1); break;
    case 2: dispatch<PolBF<3>, 3>(s, r, st, 2, 1); break;
    default: dispatch<PolBF<1>, 1>(s, r, st, 3, 1); break;
  }
}

}  // namespace arpc
