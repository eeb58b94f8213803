// One-kernel round product for the BF16 modes (ARPC_BF16, ARPC_BF16X3) on
// gfx950.  For a tile of 128 rows a workgroup computes, without C ever
// leaving the registers (Alg. 2, step 3):
//   1. C^T = Bm1 F^T on the matrix cores, Bm1 = F(S_r,:)^T, then
//      C = A(:, S_r) - (F F(S_r,:)^T) with the kernel columns evaluated from
//      the points in the accumulator layout;
//   2. G^T = Linv C^T on the matrix cores, the accumulators of step 1 serving
//      directly as the operand (see the slot permutation below);
//   3. G into F(:, k_r : k_r + s_r) (column-major FP32), into the panel-blocked
//      BF16 copy of F that the next rounds contract over, and the row norms
//      of G for the residual-diagonal update.
//
// Workgroups are persistent and walk the row tiles; each F element is read
// from HBM once per round.  Wavefront w owns 32 rows of the tile and all
// columns; its F slices are loaded straight from HBM into registers FD chunks
// ahead.  The small operands (Bm1 chunks, and in the three-product mode the
// chunks of the permuted inverse factor) stream through a two-stage LDS ring
// shared by the workgroup's wavefronts.
//
// Slot permutation.  A 16x16x32 BF16 product takes, in lane (g, n), operand
// values for contraction slots 8g .. 8g+7 of column n.  The accumulator of
// the update GEMM holds, in lane (g, n), C(row n, 16 cb + 4g + j), j < 4.  For
// the t-chunk tc of the solve (t = 32 tc .. 32 tc + 31), slot 8g + jj is
// therefore bound to t = 32 tc + 4g + jj (jj < 4, column block 2 tc) and
// t = 32 tc + 16 + 4g + jj - 4 (jj >= 4, column block 2 tc + 1); the inverse
// factor is stored with the same slot order, so the product is exact in any
// order and no lane exchange is needed.
#include <type_traits>

#include "arpc_common.h"
#include "arpc_launch.h"
#include "arpc_mfma.h"

namespace arpc {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int FNB = 2;           // 16-row tiles per wavefront
constexpr int FKC = 32;          // contraction chunk
constexpr int FCROW = 80;        // LDS bytes per staged column and plane (64 + 16 padding)
constexpr int FGROW = 64;        // global bytes per operand column and plane
constexpr int EROW = 36;         // padded row count of the store window (16-byte rows)

// Lower-triangular blocks of the permuted inverse factor: block (mt, tc)
// holds rows i = 16 mt .. 16 mt + 15 and the t-chunk tc, and is nonzero only
// if 32 tc <= 16 mt + 15.  Resident form: the blocks of row block mt follow
// those of mt - 1, each 16 rows of FCROW bytes.
__host__ __device__ constexpr int tri_row_blocks(int mt) { return (16 * mt + 15) / 32 + 1; }
__host__ __device__ constexpr int tri_base(int mt) {
  int b = 0;
  for (int m = 0; m < mt; ++m) b += tri_row_blocks(m);
  return b;
}


// Slot of contraction index t (0..31) inside a t-chunk of the solve.
__host__ __device__ inline int solve_slot(int t) {
  return 8 * ((t & 15) >> 2) + (t & 3) + ((t & 16) ? 4 : 0);
}

__device__ inline void split_hi_lo(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// FW wavefronts per workgroup.  RES: the whole lower triangle of the inverse
// factor stays in LDS for the launch (one 8-wavefront workgroup per CU), so the
// solve needs no staging; otherwise its chunks stream through the ring (two
// 4-wavefront workgroups per CU, for the three-product mode whose two planes
// do not fit).
// TAB: the arguments come from row blockIdx.y of a table of jobs (one launch
// serving several factorizations), else from the kernel argument.
template <int PASSES, int NCBT, int DX, int FD, int FW, bool RES, bool UR, bool TAB>
__global__ __launch_bounds__(64 * FW) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fused_round(
    FusedArgs a0, const RoundJob* __restrict__ tab) {
  // arguments read where they are used, as kernel arguments are (the
  // compiler may reload them instead of holding them in registers)
  auto&& a = [&]() -> decltype(auto) {
    if constexpr (TAB) return (table_row(tab).fa);
    else return (a0);
  }();
  constexpr int SPL = PASSES == 3 ? 2 : 1;
  constexpr int CP = NCBT * 16;                 // padded column count
  constexpr int NT = (NCBT + 1) / 2;            // t-chunks of the solve
  constexpr int NPASS = 1;                      // solve passes (see below)
  constexpr int STAGE = SPL * CP * FCROW;       // LDS bytes per ring stage
  constexpr int PIECES = SPL * CP * (FGROW / 16);
  constexpr int PER_T = (PIECES + 64 * FW - 1) / (64 * FW);
  constexpr int PLANE_E = PH * FKC;             // elements per plane of a blocked chunk
  constexpr int CHUNK_E = SPL * PLANE_E;
  constexpr int WC = RES ? 32 : 64;             // columns per store window
  constexpr int RING = (2 * STAGE > FW * WC * EROW * 4) ? 2 * STAGE : FW * WC * EROW * 4;
  constexpr int TRI = RES ? tri_base(NCBT) * 16 * FCROW : 0;   // resident inverse factor
  constexpr int XPS = RING + TRI;
  constexpr int YN = XPS + CP * DX * 4;         // squared norms of the accepted points
  constexpr int DUMMY = YN + CP * 4;            // 16-byte sink of surplus staging pieces
  // SEPW: the store window has its own LDS (when it fits), so no barrier
  // separates one tile's stores from the next tile's ring; with nothing to
  // contract (k_r = 0) a tile then needs no barrier at all, and the
  // wavefronts drift apart, one's stores overlapping another's arithmetic.
  constexpr int WIN = FW * WC * EROW * 4;
  constexpr bool SEPW = RES && (DUMMY + 16 + WIN <= 160 * 1024);
  constexpr int WINOFF = DUMMY + 16;
  __shared__ __attribute__((aligned(16))) unsigned char lds[SEPW ? WINOFF + WIN : DUMMY + 16];
  float* xps = (float*)(lds + XPS);
  float* yn = (float*)(lds + YN);
  // Distances: the three-product mode differences the coordinates directly;
  // the one-product mode, whose C is rounded to BF16 anyway, uses
  // |x|^2 + |y|^2 - 2 x.y with the product on the matrix cores (its FP32
  // cancellation error, about |x|^2 * 2^-23, is far below the BF16 rounding
  // of C).
  constexpr bool EXPAND = PASSES == 1;

  const RoundState* st = a.st;
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  if (s == 0) return;
  // the last column block holds accepted columns (else its update and solve
  // products are exactly zero and are skipped: the accumulators keep their
  // zeros).  The solve's skip is compiled where it leaves the register
  // allocation as it is (one product, d <= 16).
  const bool lastcb = s > 16 * (NCBT - 1);
  constexpr bool SKIP_SOLVE = PASSES == 1 && DX <= 16;
  const int64_t kr = st->k_r;
  const int64_t nk = (kr + FKC - 1) / FKC;      // contraction chunks of the update GEMM
  const int64_t N = a.N;
  constexpr int FROWS = FW * FNB * 16;           // rows per workgroup tile
  const int ntiles = (int)((N + FROWS - 1) / FROWS);
  const int d = a.d;
  const int tid0 = threadIdx.x, w = tid0 >> 6;

  // The kernel's scale folds into the points.  Every kernel here is
  // phi(sqrt(cr) r) with phi(t) = (1 + p1 t + p2 t^2) 2^(-q t) (use_r) or
  // phi(r^2) = 2^(-cr r^2) (Gaussian), so one scaled squared distance
  // e = cr |x - y|^2 is all a column needs.
  const KFast kf = ldc_any(a.kf);
  const float cr = UR ? kf.scale * kf.scale : kf.q * kf.scale;
  // accepted points in FP32, zero-padded to DX coordinates and CP columns.
  // Expanded form: r^2 = |x|^2 + |y|^2 - 2 x.y, the product on the matrix
  // cores, so the points are stored coordinate-major and scaled by -2, with
  // |y|^2 beside them; the scale cr multiplies r^2 after the cancellation
  // (exact for points on an integer grid, as in the unscaled form).  Direct
  // form: the points scaled by sqrt(cr), column-major.
  const float sxp = EXPAND ? -2.f : sqrtf(cr);
  for (int q = tid0; q < CP * DX; q += 64 * FW) {
    const int c = EXPAND ? q % CP : q / DX, t = EXPAND ? q / CP : q % DX;
    xps[q] = (c < s && t < d) ? sxp * (float)a.Xp[(int64_t)c * d + t] : 0.f;
  }
  if constexpr (EXPAND) {
    for (int c = tid0; c < CP; c += 64 * FW) {
      float n2 = 0.f;
      for (int t = 0; t < d && c < s; ++t) {
        const float y = (float)a.Xp[(int64_t)c * d + t];
        n2 = fmaf(y, y, n2);
      }
      yn[c] = n2;
    }
  }

  if constexpr (RES) {
    // the inverse factor's triangle, once per launch (ordered before its first
    // use by the barrier below, or the first barrier of the tile loop)
    for (int q = tid0; q < TRI / 16; q += 64 * FW)
      *(u4*)(lds + RING + q * 16) = *(const u4*)(a.Bm2 + (size_t)q * 16);
  }
  if constexpr (SEPW) __syncthreads();

  // ---- small-operand ring: stream position q < nk is chunk q of Bm1, then
  // (streaming form) the NT chunks of the inverse factor.  Chunks are loaded
  // into registers D positions ahead of their commit to the two-stage LDS
  // ring, so the load latency (an L2 round trip per chunk) overlaps D
  // iterations of the contraction.
  constexpr int D = RES ? FD : 1;
  const int64_t nkl = nk > 0 ? nk - 1 : 0;       // last valid chunk index
  u4 sbq[D][PER_T];
  int tid = tid0;
  auto fetch_to = [&](u4 (&sbuf)[PER_T], int64_t q) {
    const unsigned char* src;
    if constexpr (RES) src = a.Bm1 + (size_t)(q < nkl ? q : nkl) * SPL * CP * FGROW;
    else src = (q < nk) ? a.Bm1 + (size_t)q * SPL * CP * FGROW
                        : a.Bm2 + (size_t)((q - nk) % NT) * SPL * CP * FGROW;
    // every thread issues the same loads (a piece index past the stage is
    // clamped and its value dropped at the commit), so the number of loads in
    // flight is the same on every path and the waits stay exact
#pragma unroll
    for (int r = 0; r < PER_T; ++r) {
      const int o = tid + r * 64 * FW;
      sbuf[r] = *(const u4*)(src + (size_t)(o < PIECES ? o : PIECES - 1) * 16);
    }
  };
  auto commit_from = [&](const u4 (&sbuf)[PER_T], int buf) {
#pragma unroll
    for (int r = 0; r < PER_T; ++r) {
      const int o = tid + r * 64 * FW;
      const int pc = o >> 2, qq = o & 3;       // (plane, column) and 16-byte piece
      // unguarded as well: surplus pieces go to a dummy slot
      const int dst = o < PIECES ? buf * STAGE + pc * FCROW + qq * 16 : DUMMY;
      *(u4*)(lds + dst) = sbuf[r];
    }
  };

  // Operands a tile starts with: its rows' coordinates and the first D chunks
  // of Bm1 (early part), the first FD - 1 chunks of F (late part).  Where the
  // registers allow (PRE), the early part for the next tile is loaded before
  // the stores of the current one, so those loads go out ahead of the stores
  // instead of queueing behind them.
  constexpr bool PRE = NCBT <= 13;
  constexpr int XR = EXPAND ? DX / 4 : DX;
  float xr[FNB][XR];
  bf8 fr[FD][FNB][SPL];
  // F slices: rows row_w + l16 and row_w + 16 + l16 share a 256-row panel
  auto fbase = [&](int64_t row_w_, int l16_, int g_) {
    const int64_t r0 = row_w_ + l16_;
    return a.Fb + (size_t)(r0 / PH) * a.nkc * CHUNK_E + (size_t)(r0 % PH) * FKC + 8 * g_;
  };
  auto loadF = [&](bf8 (&f)[FNB][SPL], const __bf16* rb, int64_t ch) {
#pragma unroll
    for (int nb = 0; nb < FNB; ++nb)
#pragma unroll
      for (int pl = 0; pl < SPL; ++pl)
        f[nb][pl] = *(const bf8*)(rb + (size_t)ch * CHUNK_E + pl * PLANE_E + nb * 16 * FKC);
  };
  auto prologue_early = [&](int tile_) {
    const int lane_ = tid & 63, l16_ = lane_ & 15, g_ = lane_ >> 4;
    const int64_t row_w_ = (int64_t)tile_ * FROWS + w * (FNB * 16);
    // this lane's rows (tiles nb = 0, 1): row_w + 16 nb + l16.  Expanded
    // form: coordinates 4 ks + g only, the B operand of the distance product
    // (lane (g, n) holds B(k = g, n)); direct form: all coordinates, scaled.
#pragma unroll
    for (int nb = 0; nb < FNB; ++nb) {
      int64_t r = row_w_ + nb * 16 + l16_;
      if (r >= N) r = N - 1;
#pragma unroll
      for (int t = 0; t < XR; ++t) {
        const int tt = EXPAND ? 4 * t + g_ : t;
        xr[nb][t] = (tt < d) ? (EXPAND ? 1.f : sxp) * (float)a.X[r * d + tt] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < D; ++u) fetch_to(sbq[u], u);
  };
  auto prologue_late = [&](const __bf16* rb_) {
#pragma unroll
    for (int u = 0; u < FD - 1; ++u) loadF(fr[u], rb_, u < nkl ? u : nkl);
  };
  if (PRE && (int)blockIdx.x < ntiles) {
    tid = tid0;
    asm volatile("" : "+v"(tid));
    prologue_early(blockIdx.x);
  }

  // tiles are dealt to the persistent workgroups in turn
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // Lane-dependent values are re-derived in every tile: hoisted out of the
    // loop they would stay live across it and spill.
    tid = tid0;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, l16 = lane & 15, g = lane >> 4;
    const int64_t row_w = (int64_t)tile * FROWS + w * (FNB * 16);

    f4 acc[FNB][NCBT];
#pragma unroll
    for (int nb = 0; nb < FNB; ++nb)
#pragma unroll
      for (int cb = 0; cb < NCBT; ++cb) acc[nb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    const __bf16* rb = fbase(row_w, l16, g);
    if (!PRE) prologue_early(tile);
    prologue_late(rb);
    // ---- 1. update GEMM.  The loop body is straight-line in its loads: each
    // iteration fetches the next small-operand chunk and loads the F chunk
    // FD - 1 ahead (clamped to the last chunk near the end; the surplus loads
    // are never consumed); only the products are guarded.  The
    // load counter is in-order, so the fetch goes first: the wait before its
    // commit leaves the F loads in flight.
    if (!SEPW || nk > 0) {   // uniform
      commit_from(sbq[0], 0);
      __syncthreads();
    }

    for (int64_t ch0 = 0; ch0 < nk; ch0 += FD) {
#pragma unroll
      for (int u = 0; u < FD; ++u) {
        const int64_t ch = ch0 + u;
        // slot u % D held chunk ch, committed at the end of the previous
        // iteration; it now receives chunk ch + D
        fetch_to(sbq[u % D], (D == 1 && ch + 1 > nk) ? nk : ch + D);
        loadF(fr[(u + FD - 1) % FD], rb, ch + FD - 1 < nkl ? ch + FD - 1 : nkl);
        if (ch < nk) {
          const unsigned char* L = lds + (ch & 1) * STAGE + l16 * FCROW + g * 16;
          // operand reads PD - 1 column blocks ahead of the products: enough
          // LDS reads in flight to cover their latency, without holding all
          // NCBT operand slices in registers
          constexpr int PD = (PASSES == 3 || NCBT > 13) ? 2 : 4;
          bf8 ap[PD], alp[PD];
#pragma unroll
          for (int j = 0; j < PD - 1 && j < NCBT; ++j) {
            ap[j] = *(const bf8*)(L + j * 16 * FCROW);
            if constexpr (PASSES == 3) alp[j] = *(const bf8*)(L + CP * FCROW + j * 16 * FCROW);
          }
#pragma unroll
          for (int cb = 0; cb < NCBT; ++cb) {
            if (cb + PD - 1 < NCBT) {
              ap[(cb + PD - 1) % PD] = *(const bf8*)(L + (cb + PD - 1) * 16 * FCROW);
              if constexpr (PASSES == 3) alp[(cb + PD - 1) % PD] = *(const bf8*)(L + CP * FCROW + (cb + PD - 1) * 16 * FCROW);
            }
            const bf8 ah = ap[cb % PD];
            bf8 al;
            if constexpr (PASSES == 3) al = alp[cb % PD];
            if (cb + 1 < NCBT || lastcb)
#pragma unroll
            for (int nb = 0; nb < FNB; ++nb) {
              acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr[u][nb][0], acc[nb][cb], 0, 0, 0);
              if constexpr (PASSES == 3) {
                acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, fr[u][nb][1], acc[nb][cb], 0, 0, 0);
                acc[nb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, fr[u][nb][0], acc[nb][cb], 0, 0, 0);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // unguarded: past the last chunk the fetch repeats the first chunk of
        // the inverse factor (already committed), and no product reads the
        // buffer written here
        commit_from(sbq[(u + 1) % D], (ch + 1) & 1);
        __syncthreads();
      }
    }

    // |x|^2 of this lane's rows (expanded form): the partial sums of the
    // four lanes that hold a row's coordinates, added in the same order in
    // each of them
    float xa[FNB];
    if constexpr (EXPAND) {
#pragma unroll
      for (int nb = 0; nb < FNB; ++nb) {
        float n2 = 0.f;
#pragma unroll
        for (int t = 0; t < XR; ++t) n2 = fmaf(xr[nb][t], xr[nb][t], n2);
        n2 += __shfl_xor(n2, 16, 64);
        n2 += __shfl_xor(n2, 32, 64);
        xa[nb] = n2;
      }
    }
    // ---- kernel columns and solve.  (A pass per 16-row tile would halve the
    // live solve state but streams the inverse factor twice; with this
    // compiler it spilled more, so both tiles are solved in one pass.)
    f4 gacc[FNB][NCBT];
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      constexpr int NPB = FNB / NPASS;                // row tiles per pass
      const int nb0 = pass * NPB;
      // kernel columns: C = kappa(x_row, x_c) - acc as the BF16 operand slices
      // of the solve (slot order above).  Columns c >= s hold finite values
      // (zero points, zero update) that meet only zero inverse-factor
      // entries, so they are not masked.
      bf8 ch_[NPB][NT][SPL];
      // phi of four scaled squared distances
      auto phi4 = [&](f4 e) __attribute__((always_inline)) {
        f4 k;
        if constexpr (UR) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float t = __builtin_amdgcn_sqrtf(fmaxf(e[j], 0.f));
            k[j] = fmaf(fmaf(kf.p2, t, kf.p1), t, 1.f) * __builtin_amdgcn_exp2f(-kf.q * t);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) k[j] = __builtin_amdgcn_exp2f(-fmaxf(e[j], 0.f));
        }
        return k;
      };
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        f8 cv[NPB];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int cb = 2 * tc + half;
          if (cb < NCBT) {
            if constexpr (EXPAND) {
              // r^2 = |x|^2 + |y|^2 - 2 x.y: lane (g, n) of a 16x16x4 FP32
              // product holds (column 16 cb + 4 g + j, row n), the layout of
              // the update accumulators
              const f4 y4 = *(const f4*)(yn + cb * 16 + 4 * g);
#pragma unroll
              for (int ib = 0; ib < NPB; ++ib) {
                f4 e4 = y4 + xa[nb0 + ib];
#pragma unroll
                for (int ks = 0; ks < XR; ++ks)
                  e4 = __builtin_amdgcn_mfma_f32_16x16x4f32(xps[(4 * ks + g) * CP + cb * 16 + l16], xr[nb0 + ib][ks],
                                                           e4, 0, 0, 0);
                const f4 k4 = phi4(cr * e4) - acc[nb0 + ib][cb];
#pragma unroll
                for (int j = 0; j < 4; ++j) cv[ib][4 * half + j] = k4[j];
              }
            } else {
              f4 e4[NPB];
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                const int c = cb * 16 + 4 * g + j;
                float xp[DX];
#pragma unroll
                for (int t = 0; t < DX; ++t) xp[t] = xps[c * DX + t];
#pragma unroll
                for (int ib = 0; ib < NPB; ++ib) {
                  float e = 0.f;
#pragma unroll
                  for (int t = 0; t < DX; ++t) {
                    const float df = xr[nb0 + ib][t] - xp[t];
                    e = fmaf(df, df, e);
                  }
                  e4[ib][j] = e;
                }
              }
#pragma unroll
              for (int ib = 0; ib < NPB; ++ib) {
                const f4 k4 = phi4(e4[ib]) - acc[nb0 + ib][cb];
#pragma unroll
                for (int j = 0; j < 4; ++j) cv[ib][4 * half + j] = k4[j];
              }
            }
          } else {
#pragma unroll
            for (int ib = 0; ib < NPB; ++ib)
#pragma unroll
              for (int j = 0; j < 4; ++j) cv[ib][4 * half + j] = 0.f;
          }
        }
#pragma unroll
        for (int ib = 0; ib < NPB; ++ib) {
          ch_[ib][tc][0] = __builtin_convertvector(cv[ib], bf8);
          if constexpr (SPL == 2)
            ch_[ib][tc][1] = __builtin_convertvector(cv[ib] - __builtin_convertvector(ch_[ib][tc][0], f8), bf8);
        }
      }
      // Materialise the operand slices here: sunk into the solve loop, their
      // computation would keep the update-GEMM accumulators alive beside the
      // solve accumulators.
#pragma unroll
      for (int ib = 0; ib < NPB; ++ib)
#pragma unroll
        for (int tc = 0; tc < NT; ++tc)
#pragma unroll
          for (int pl = 0; pl < SPL; ++pl) asm volatile("" : "+v"(ch_[ib][tc][pl]));

      // ---- 2. solve: G^T = Linv C^T over the lower-triangular blocks
#pragma unroll
      for (int ib = 0; ib < NPB; ++ib)
#pragma unroll
        for (int mt = 0; mt < NCBT; ++mt) gacc[nb0 + ib][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tc = 0; tc < NT; ++tc) {
        const int64_t q = nk + pass * NT + tc;
        const bool more = !RES && (tc + 1 < NT || pass + 1 < NPASS);
        if (more) fetch_to(sbq[0], q + 1);
        const unsigned char* L = lds + (q & 1) * STAGE;
#pragma unroll
        for (int mt = 0; mt < NCBT; ++mt) {
          if (32 * tc <= 16 * mt + 15 && (!SKIP_SOLVE || mt + 1 < NCBT || lastcb)) {
            bf8 ah, al;
            if constexpr (RES) {
              ah = *(const bf8*)(lds + RING + (tri_base(mt) + tc) * 16 * FCROW + l16 * FCROW + g * 16);
            } else {
              ah = *(const bf8*)(L + (mt * 16 + l16) * FCROW + g * 16);
              if constexpr (PASSES == 3) al = *(const bf8*)(L + CP * FCROW + (mt * 16 + l16) * FCROW + g * 16);
            }
#pragma unroll
            for (int ib = 0; ib < NPB; ++ib) {
              f4& gq = gacc[nb0 + ib][mt];
              gq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ch_[ib][tc][0], gq, 0, 0, 0);
              if constexpr (PASSES == 3) {
                gq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ch_[ib][tc][1], gq, 0, 0, 0);
                gq = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, ch_[ib][tc][0], gq, 0, 0, 0);
              }
            }
          }
        }
        if constexpr (!RES) {
          if (more) commit_from(sbq[0], (q + 1) & 1);
          __syncthreads();
        }
      }
    }

    // ---- 3. row norms, the blocked copy, then F through a per-wavefront LDS
    // window.  Lane (g, l16) holds G(row_w + 16 nb + l16, i) for
    // i = 16 mt + 4 g + j; G(:, i) is exactly zero for s <= i < CP (zero rows
    // of the inverse factor).  Norms: FP32 sums over a lane's 4 NCBT entries
    // (relative error a few 2^-24, far below the BF16 rounding of G), then
    // over the four lanes of a row.
#pragma unroll
    for (int nb = 0; nb < FNB; ++nb) {
      float g2 = 0.f;
#pragma unroll
      for (int mt = 0; mt < NCBT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) g2 = fmaf(gacc[nb][mt][j], gacc[nb][mt][j], g2);
      g2 += __shfl_xor(g2, 16, 64);
      g2 += __shfl_xor(g2, 32, 64);
      const int64_t row = row_w + nb * 16 + l16;
      if (row < N && g == 0) a.P[row] = (double)g2;
    }
    if (PRE && tile + (int)gridDim.x < ntiles) prologue_early(tile + gridDim.x);
    // Blocked BF16 copy, 8-byte stores straight from the accumulators.  Its
    // columns kr - m .. are cut into groups of four (m = kr mod 4, so a group
    // never crosses a 32-column chunk): lane (g, l16) of group mt writes
    // columns kr - m + 16 mt + 4 g .. + 3, which hold G(:, i) for
    // i = 16 mt + 4 g - m .. + 3: its own entries j < 4 - m, and the last m
    // entries of the lane before it (lane g - 1, or lane g = 3 of group
    // mt - 1), fetched with one lane permutation per 32-bit word.  The
    // groups run on past CP as zeros up to the end of the last chunk, which
    // the next round's contraction reads whole.  The first group of a round
    // starts m columns inside the previous round's: that lane writes only its
    // own 4 - m values.
    {
      const int m = (int)(kr & 3);
      const int64_t zend = (kr + s + FKC - 1) / FKC * FKC;
      const int sh = 16 * m;
      const int src = (lane + 48) & 63;                  // lane g - 1 (mod 4), same l16
#pragma unroll
      for (int nb = 0; nb < FNB; ++nb) {
        const int64_t row = row_w + nb * 16 + l16;
        __bf16* prow = a.Fbw + (row / PH) * a.nkc * (int64_t)CHUNK_E + (row % PH) * FKC;
        uint64_t tprev[SPL];
#pragma unroll
        for (int pl = 0; pl < SPL; ++pl) tprev[pl] = 0;
#pragma unroll
        for (int mt = 0; mt < NCBT + 3; ++mt) {
          const int64_t a0 = kr - m + 16 * mt + 4 * g;
          __bf16* p = prow + (a0 / FKC) * (int64_t)CHUNK_E + a0 % FKC;
          const bool ok = row < N && a0 < zend;
          const bool first = mt == 0 && g == 0 && m != 0;
#pragma unroll
          for (int pl = 0; pl < SPL; ++pl) {
            uint64_t v = 0;
            if (mt < NCBT) {
              const f4 gv = gacc[nb][mt < NCBT ? mt : 0];
              __bf16 h[4];   // plane 0: BF16 of G; plane 1: BF16 of the remainder
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                h[j] = (__bf16)gv[j];
                if (pl == 1) h[j] = (__bf16)(gv[j] - (float)h[j]);
              }
              v = (uint64_t)__builtin_bit_cast(unsigned short, h[0]) |
                  ((uint64_t)__builtin_bit_cast(unsigned short, h[1]) << 16) |
                  ((uint64_t)__builtin_bit_cast(unsigned short, h[2]) << 32) |
                  ((uint64_t)__builtin_bit_cast(unsigned short, h[3]) << 48);
            }
            const unsigned lo32 = __shfl((unsigned)v, src, 64), hi32 = __shfl((unsigned)(v >> 32), src, 64);
            const uint64_t t = (uint64_t)lo32 | ((uint64_t)hi32 << 32);
            const uint64_t pv = g == 0 ? tprev[pl] : t;
            tprev[pl] = t;
            const uint64_t out = m ? (v << sh) | (pv >> (64 - sh)) : v;
            __bf16* pp = p + pl * PLANE_E;
            if (ok) {
              if (first) {
#pragma unroll
                for (int jj = 1; jj < 4; ++jj)
                  if (jj >= m) pp[jj] = __builtin_bit_cast(__bf16, (unsigned short)(out >> (16 * jj)));
              } else {
                *(uint64_t*)pp = out;
              }
            }
          }
        }
      }
    }
    // E[col][row]: WC columns x 32 rows of this wavefront (its own area with
    // SEPW, else the ring area: no wavefront reads the ring after the last
    // barrier of the contraction)
    float* E = (float*)(lds + (SEPW ? WINOFF : 0)) + w * (WC * EROW);
    const int nrows = (N - row_w) < (FNB * 16) ? (int)(N - row_w) : FNB * 16;
    const bool vec_cols = (N & 3) == 0;          // 16-byte aligned columns of F
#pragma unroll
    for (int w0 = 0; w0 < CP; w0 += WC) {
#pragma unroll
      for (int mt = w0 / 16; mt < w0 / 16 + WC / 16 && mt < NCBT; ++mt)
#pragma unroll
        for (int nb = 0; nb < FNB; ++nb)
#pragma unroll
          for (int j = 0; j < 4; ++j) E[(mt * 16 - w0 + 4 * g + j) * EROW + nb * 16 + l16] = gacc[nb][mt][j];
      int wv = s - w0;
      if (wv > WC) wv = WC;
      // F, column-major: 4 consecutive rows per lane (16-byte stores), or one
      // row per lane when the columns are not 16-byte aligned
      if (vec_cols && nrows == FNB * 16) {
        for (int cc = lane >> 3; cc < wv; cc += 8) {
          const int r4 = 4 * (lane & 7);
          *(f4*)(a.Fu + (kr + w0 + cc) * N + row_w + r4) = *(const f4*)(E + cc * EROW + r4);
        }
      } else {
        for (int cc = lane >> 5; cc < wv; cc += 2) {
          const int rl = lane & 31;
          if (rl < nrows) a.Fu[(kr + w0 + cc) * N + row_w + rl] = E[cc * EROW + rl];
        }
      }
    }
    if constexpr (!SEPW) __syncthreads();   // the window area is the ring of the next tile
  }
}

// Bm1 chunk j, column c: the blocked slice of F at row S_r(c) (zero for c >=
// s), 16-byte pieces taken by virtual workgroup vb of vg.
template <int SPL>
__device__ __attribute__((always_inline)) inline void bm1_range(ConstRoundJob& RJ, int s, int64_t kr, int vb, int vg) {
  const __bf16* __restrict__ Fb = (const __bf16*)RJ.Fb;
  const int64_t nkc = RJ.nkc;
  const int64_t* __restrict__ props = RJ.props;
  const int32_t* __restrict__ acc = RJ.acc;
  const int CP = RJ.CP;
  unsigned char* __restrict__ Bm1 = RJ.Bm1;
  const int64_t nk = (kr + FKC - 1) / FKC;
  const int64_t per_chunk = (int64_t)SPL * CP * 4;  // 16-byte pieces
  for (int64_t o = (int64_t)vb * 256 + threadIdx.x; o < nk * per_chunk; o += (int64_t)vg * 256) {
    const int64_t j = o / per_chunk;
    const int rem = (int)(o % per_chunk);
    const int plane = rem / (CP * 4), c = (rem / 4) % CP, q = rem & 3;
    u4 v = u4{0, 0, 0, 0};
    if (c < s) {
      const int64_t row = props[acc[c]];
      v = *(const u4*)(Fb + (((row / PH) * nkc + j) * SPL + plane) * (int64_t)(PH * FKC) + (row % PH) * FKC + 8 * q);
    }
    *(u4*)(Bm1 + (size_t)o * 16) = v;
  }
}

// Inverse of the s x s lower factor L (read from H through the accepted
// indices), column t by one workgroup: block forward substitution from the
// blocks' inverses that the tiled rejection kernel leaves in H (b <= 256 here),
// then Linv(i, t) stored at chunk t / 32, slot solve_slot(t % 32), column i
// (zero outside i, t < s and below the diagonal).
template <int SPL, bool RES>
__device__ __attribute__((always_inline)) inline void linv_column_to_bm2(ConstRoundJob& RJ, int s, int c) {
  const int CP = RJ.CP;
  unsigned char* __restrict__ Bm2 = RJ.Bm2;
  const int tid = threadIdx.x;
  __shared__ double x[256];
  __shared__ double xp[256];   // proposal-indexed column
  __shared__ double ys[128];
  if (c < s) {   // uniform
    linv_blocks_ahead<4>(RJ.H, RJ.acc, RJ.b, s, c, tid, xp, ys);
    for (int i = tid; i < s; i += 256) x[i] = xp[RJ.acc[i]];
  }
  __syncthreads();
  const int tc = c / FKC, slot = solve_slot(c % FKC);
  if constexpr (RES) {
    // rows 32 tc .. CP - 1 of the blocks (i / 16, tc) of the resident triangle
    for (int i = FKC * tc + tid; i < CP; i += 256) {
      const double v = (c < s && i >= c && i < s) ? x[i] : 0.0;
      unsigned char* base = Bm2 + (size_t)(tri_base(i / 16) + tc) * 16 * FCROW + (size_t)(i % 16) * FCROW + slot * 2;
      *(__bf16*)base = (__bf16)(float)v;
    }
  } else {
    for (int i = tid; i < CP; i += 256) {
      const double v = (c < s && i >= c && i < s) ? x[i] : 0.0;
      __bf16 hi, lo;
      split_hi_lo((float)v, hi, lo);
      unsigned char* base = Bm2 + (size_t)tc * SPL * CP * FGROW + (size_t)i * FGROW + slot * 2;
      *(__bf16*)base = hi;
      if (SPL == 2) *(__bf16*)(base + (size_t)CP * FGROW) = lo;
    }
  }
}

// The round product's operands in one launch, in three ranges of workgroups:
// [0, nl) the inverse factor (a column each), [nl, nl + nb) the Bm1 chunks,
// [nl + nb, ...) the accepted points.  The three read only the rejection
// step's outputs and write disjoint buffers.
template <int SPL, bool RES, bool TAB>
__global__ __launch_bounds__(256) void k_fused_prep(RoundJob j0, const RoundJob* __restrict__ tab, int nl, int nb,
                                                    int nx) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int v = blockIdx.x;
  if (v < nl) {
    if (v < RJ.nt * FKC) linv_column_to_bm2<SPL, RES>(RJ, s, v);   // uniform
  } else if (v < nl + nb) {
    bm1_range<SPL>(RJ, s, st->k_r, v - nl, nb);
  } else {
    prep_xp_range(RJ, s, v - nl - nb, nx);
  }
}

// Column-block counts with a compiled instance.
constexpr int kNcbt[] = {2, 4, 8, 13, 16};

int ncbt_for(int b) {
  const int need = (b + 15) / 16;
  for (int v : kNcbt)
    if (v >= need) return v;
  return -1;
}

// One-plane BF16: resident inverse factor, one 8-wavefront workgroup per CU.
// Three-product BF16: streamed inverse factor, two 4-wavefront workgroups per CU.
template <int PASSES>
struct FusedShape {
  static constexpr bool RES = PASSES == 1;
  static constexpr int FW = RES ? 8 : 4;
  static constexpr int PER_CU = RES ? 1 : 2;
  // F chunks in flight: the three-product mode spends three times the matrix
  // time per chunk, so one chunk ahead hides as much latency
  static constexpr int FD = PASSES == 3 ? 2 : 4;
};

template <int PASSES, int NCBT, int DX, bool TAB>
void launch_fused_t(hipStream_t s, const FusedArgs& a, const RoundJob* tab, int n, int grid) {
  using SH = FusedShape<PASSES>;
  if (a.kf.use_r)
    hipLaunchKernelGGL((k_fused_round<PASSES, NCBT, DX, SH::FD, SH::FW, SH::RES, true, TAB>), dim3(grid, n),
                       dim3(64 * SH::FW), 0, s, a, tab);
  else
    hipLaunchKernelGGL((k_fused_round<PASSES, NCBT, DX, SH::FD, SH::FW, SH::RES, false, TAB>), dim3(grid, n),
                       dim3(64 * SH::FW), 0, s, a, tab);
}

template <int PASSES, int NCBT, bool TAB>
void launch_fused_d(hipStream_t s, int dx, const FusedArgs& a, const RoundJob* tab, int n, int grid) {
  if (dx <= 8) {
    launch_fused_t<PASSES, NCBT, 8, TAB>(s, a, tab, n, grid);
  } else if (dx <= 16) {
    launch_fused_t<PASSES, NCBT, 16, TAB>(s, a, tab, n, grid);
  } else {
    // d <= 32: the one-product mode with at most 13 column blocks (its LDS
    // holds the accepted points' 32 coordinates beside the resident inverse
    // factor).  The three-product mode differences coordinates directly and
    // keeps the two-kernel round product there.
    if constexpr (PASSES == 1 && NCBT <= 13) launch_fused_t<PASSES, NCBT, 32, TAB>(s, a, tab, n, grid);
  }
}

template <int PASSES, bool TAB>
void launch_fused_p(hipStream_t s, int ncbt, int dx, const FusedArgs& a, const RoundJob* tab, int n, int grid) {
  switch (ncbt) {
    case 2: launch_fused_d<PASSES, 2, TAB>(s, dx, a, tab, n, grid); break;
    case 4: launch_fused_d<PASSES, 4, TAB>(s, dx, a, tab, n, grid); break;
    case 8: launch_fused_d<PASSES, 8, TAB>(s, dx, a, tab, n, grid); break;
    case 13: launch_fused_d<PASSES, 13, TAB>(s, dx, a, tab, n, grid); break;
    default: launch_fused_d<PASSES, 16, TAB>(s, dx, a, tab, n, grid); break;
  }
}

template <int PASSES>
int fused_rows() {
  using SH = FusedShape<PASSES>;
  return SH::FW * FNB * 16;
}

}  // namespace

int fused_ncbt(int prec, int b) {
  if (prec != 2 && prec != 3) return -1;
  return ncbt_for(b);
}

size_t fused_operand_bytes(int prec, int64_t kmax, int b) {
  const int ncbt = fused_ncbt(prec, b);
  if (ncbt < 0) return 0;
  const int spl = prec == 2 ? 2 : 1;
  const int64_t cp = 16 * ncbt;
  const int64_t chunks = (kmax + FKC - 1) / FKC;
  const int64_t nt = (ncbt + 1) / 2;
  const int64_t m = chunks > nt ? chunks : nt;
  const size_t streamed = (size_t)m * spl * cp * FGROW;
  const size_t resident = (size_t)tri_base(ncbt) * 16 * FCROW;   // one-plane mode
  return streamed > resident ? streamed : resident;
}

FusedArgs fused_args_of(int prec, const FusedRound& r, const RoundState* st) {
  const int rows = prec == 2 ? fused_rows<3>() : fused_rows<1>();
  return FusedArgs{(const __bf16*)r.Fb, r.nkc, r.N, r.Bm1, r.Bm2, r.X, r.d, r.Xp, kfast_of(r.kp), (float*)r.F,
                   (__bf16*)r.Fb, r.P, st, (int)((r.N + rows - 1) / rows)};
}

int fused_grid_of(int prec, const FusedArgs& a, int grid2) {
  const int per_cu = prec == 2 ? FusedShape<3>::PER_CU : FusedShape<1>::PER_CU;
  int g = grid2 / 2 * per_cu;   // grid2 is two per compute unit
  return g > a.ntiles ? a.ntiles : (g < 1 ? 1 : g);
}

void launch_fused_prep_tab(hipStream_t s, int prec, const RoundJob* tab, int n, int ncbt, int64_t bd) {
  const int nl = (ncbt + 1) / 2 * FKC, nb = 512, nx = (int)prep_xp_blocks(bd);
  const dim3 grid((unsigned)(nl + nb + nx), (unsigned)n);
  if (prec == 2)
    hipLaunchKernelGGL((k_fused_prep<2, false, true>), grid, dim3(256), 0, s, RoundJob{}, tab, nl, nb, nx);
  else
    hipLaunchKernelGGL((k_fused_prep<1, true, true>), grid, dim3(256), 0, s, RoundJob{}, tab, nl, nb, nx);
}

void launch_fused_round_tab(hipStream_t s, int prec, int ncbt, int d, const FusedArgs& any, const RoundJob* tab,
                            int n, int grid) {
  if (prec == 2) launch_fused_p<3, true>(s, ncbt, d, any, tab, n, grid);
  else launch_fused_p<1, true>(s, ncbt, d, any, tab, n, grid);
}

}  // namespace arpc
