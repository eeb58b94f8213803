// Round kernels of accelerated RPCholesky (Alg. 2, Section 2.3) other than the
// two N-sized GEMMs: residual-diagonal set-up and update, proposal draws,
// gathers at the proposals, the b x b residual submatrix, RejectionSample-
// Submatrix (Alg. 1, Section 2.2) in one workgroup, the triangular inverse and
// the end-of-round bookkeeping.  Every kernel reads the device-resident
// RoundState and returns at once when the run has stopped, so the host can
// enqueue rounds without synchronising.
#include <type_traits>

#include "arpc_common.h"
#include "arpc_launch.h"
#include "arpc_mfma.h"

namespace arpc {

// ----------------------------------------------------------------- reductions
// Deterministic block sum (fixed tree order) of one double per thread.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Inclusive prefix sum across a 64-wide wavefront (fixed order).
__device__ inline double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// -------------------------------------------------------------- initialisation
// u = diag A = kappa(0) (Alg. 2, initialisation), per-chunk sums of u, and a
// scan of X for non-finite coordinates.
__global__ __launch_bounds__(CHUNK) void k_init(double* __restrict__ u, double* __restrict__ csum,
                                                const double* __restrict__ X, int64_t N, int d,
                                                KParams kp, RoundState* st) {
  __shared__ double sh[CHUNK];
  const int64_t j0 = (int64_t)blockIdx.x * CHUNK, j = j0 + threadIdx.x;
  double v = 0.0;
  if (j < N) {
    v = kappa_r2(0.0, kp);
    u[j] = v;
  }
  // nonfinite coordinates: this workgroup's rows are one contiguous range of
  // X, read with consecutive threads on consecutive values
  {
    const int64_t q0 = j0 * d, q1 = (j0 + CHUNK < N ? j0 + CHUNK : N) * (int64_t)d;
    bool bad = false;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += CHUNK) bad |= !isfinite(X[q]);
    if (bad) atomicOr(&st->nonfinite, 1);
  }
  const double s = block_sum<CHUNK>(v, sh);
  if (threadIdx.x == 0) csum[blockIdx.x] = s;
}

// The FP8 mode's point set: each coordinate rounded to the nearest value of
// the OCP FP8 e4m3 format (sign, 4 exponent bits with bias 7, 3 fraction
// bits: normal values (1 + f/8) 2^e for e = -6 .. 8, subnormal steps of
// 2^-9, largest finite value 448), ties to the even fraction, saturating to
// +-448 beyond it; non-finite coordinates pass through unchanged (the
// finiteness scan then reports them).  Stored as FP64 (exact).
__device__ inline double round_e4m3(double x) {
  if (!isfinite(x)) return x;
  const double a = fabs(x);
  if (a >= 448.0) return copysign(448.0, x);
  int e;
  (void)frexp(a, &e);                       // a in [2^(e-1), 2^e), or a = 0
  const int ex = e - 1 < -6 ? -6 : e - 1;   // binade of a; subnormals share the spacing of 2^-6
  return copysign(ldexp(rint(ldexp(a, 3 - ex)), ex - 3), x);   // 8 steps per binade, rint: ties to even
}

__global__ __launch_bounds__(256) void k_round_e4m3(const double* __restrict__ X, double* __restrict__ Xq,
                                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    Xq[i] = round_e4m3(X[i]);
}

// The FP8 mode's setup in one pass over the points when d % 4 == 0: each row
// rounded to e4m3 and stored in FP64, its codes packed four to a word with the
// FP32 squared norm of the rounded row (the operands of the distances on the
// FP8 matrix cores, summed in the same order as k_pack_e4m3), and any
// non-finite coordinate flagged in the round state, so the initialisation
// scans nothing.  One wavefront per row.
__global__ __launch_bounds__(256) void k_round_pack_e4m3(const double* __restrict__ X, int64_t N, int d,
                                                         double* __restrict__ Xq, unsigned* __restrict__ X8,
                                                         float* __restrict__ xn, RoundState* st) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  const int dw = d / 4;
  const double* x = X + row * d;
  double* xq = Xq + row * d;
  float s = 0.f;
  bool bad = false;
  for (int q = lane; q < dw; q += 64) {
    double v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double a = x[4 * q + j];
      bad |= !isfinite(a);
      v[j] = round_e4m3(a);
      xq[4 * q + j] = v[j];
    }
    int pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v[0], (float)v[1], 0, false);
    pk = __builtin_amdgcn_cvt_pk_fp8_f32((float)v[2], (float)v[3], pk, true);
    X8[row * dw + q] = (unsigned)pk;
    s += (float)v[0] * (float)v[0] + (float)v[1] * (float)v[1] + (float)v[2] * (float)v[2] + (float)v[3] * (float)v[3];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) xn[row] = s;
  if (__ballot(bad) != 0 && lane == 0) atomicOr(&st->nonfinite, 1);
}

// Chunk sums of a residual diagonal u given by the caller (the squared column
// norms in the QR method).
__global__ __launch_bounds__(CHUNK) void k_chunk_sums(const double* __restrict__ u, int64_t N,
                                                      double* __restrict__ csum) {
  __shared__ double sh[CHUNK];
  const int64_t j = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  const double t = block_sum<CHUNK>(j < N ? u[j] : 0.0, sh);
  if (threadIdx.x == 0) csum[blockIdx.x] = t;
}

// trace(A) from the chunk sums, and the initial round state.
__global__ __launch_bounds__(1024) void k_init_state(const double* __restrict__ csum, int64_t nchunks,
                                                     RoundState* st) {
  __shared__ double sh[1024];
  double v = 0.0;
  for (int64_t c = threadIdx.x; c < nchunks; c += 1024) v += csum[c];
  const double t = block_sum<1024>(v, sh);
  if (threadIdx.x == 0) {
    st->trace_A = t;
    st->T = t;
    st->k_r = 0;
    st->round = 0;
    st->proposals = 0;
    st->s_r = 0;
    st->status = st->nonfinite ? ST_EARLY : ST_RUNNING;
  }
}

// ------------------------------------------------------------------- proposals
// Inclusive prefix of the chunk sums in a fixed order (one workgroup), the
// residual trace T = sum(u) as its last value, and the early stop when T <= 0.
template <bool TAB>
__global__ __launch_bounds__(1024) void k_scan_chunks(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const double* __restrict__ csum = RJ.csum;
  const int64_t nchunks = RJ.nchunks;
  double* __restrict__ cpre = RJ.cpre;
  const int b = RJ.b;
  const Unif un = ldc(RJ.un);
  RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  __shared__ double wsum[16];
  __shared__ int64_t lastpos_sh[1024];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (un.U && 2 * (int64_t)b * (st->round + 1) > un.nU) {
    __syncthreads();
    if (tid == 0) st->status = ST_NOUNIF;
    return;
  }
  double base = 0.0;
  int64_t lastpos = -1;
  for (int64_t c0 = 0; c0 < nchunks; c0 += 1024) {
    const int64_t c = c0 + tid;
    const double v = (c < nchunks) ? csum[c] : 0.0;
    const double incl = wave_incl_scan(v);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    double woff = 0.0, tot = 0.0;
    for (int q = 0; q < 16; ++q) {
      if (q < w) woff += wsum[q];
      tot += wsum[q];
    }
    if (c < nchunks) {
      cpre[c] = base + (woff + incl);
      if (v > 0.0) lastpos = c;
    }
    base += tot;
    __syncthreads();
  }
  lastpos_sh[tid] = lastpos;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s && lastpos_sh[tid + s] > lastpos_sh[tid]) lastpos_sh[tid] = lastpos_sh[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    // base equals cpre[nchunks-1]: the segment totals were added in the same order
    st->T = base;
    st->lastpos = (int32_t)lastpos_sh[0];
    if (!(base > 0.0) || lastpos_sh[0] < 0) st->status = ST_EARLY;
  }
}

// Alg. 2 step 1: b i.i.d. draws from u / sum(u).  Draw l (uniform word
// 2br + l) is the smallest j whose running sum exceeds U_l * T: a binary
// search over the chunk prefix, then a wavefront scan inside the chunk.  An
// index with u_j = 0 is never drawn; if rounding leaves no crossing, the last
// index with u_j > 0 (in the last positive chunk) is taken.
constexpr int PROPOSE_WAVES = 4;

// Draw l inside chunk c: the smallest j whose running sum (base + the sums of
// the chunk's entries before it) exceeds x, else the last index with u_j > 0
// in the chunk.  One wavefront; lane 0 stores props[l].
__device__ __attribute__((always_inline)) inline void draw_in_chunk(const double* __restrict__ u, int64_t N, int64_t c,
                                                                    double base, double x, int lane, int l,
                                                                    int64_t* __restrict__ props) {
  // lane l owns elements [16 lane, 16 lane + 16) of the chunk
  const int64_t e0 = c * CHUNK + 16 * lane;
  double v[16];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    v[i] = (e0 + i < N) ? u[e0 + i] : 0.0;
    s += v[i];
  }
  const double incl = wave_incl_scan(s);
  double excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 0.0;
  double run = base + excl;
  int hit = -1, lastp = -1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    run += v[i];
    if (hit < 0 && v[i] > 0.0 && run > x) hit = i;
    if (v[i] > 0.0) lastp = i;
  }
  const uint64_t hits = __ballot(hit >= 0);
  int64_t pick;
  if (hits) {
    const int fl = __ffsll((unsigned long long)hits) - 1;
    const int hi_ = __shfl(hit, fl, 64);
    pick = c * CHUNK + 16 * fl + hi_;
  } else {
    const uint64_t pos = __ballot(lastp >= 0);
    if (pos) {
      const int ll = 63 - __clzll((unsigned long long)pos);
      const int li = __shfl(lastp, ll, 64);
      pick = c * CHUNK + 16 * ll + li;
    } else {
      pick = c * CHUNK;  // unreachable for a chunk with a positive sum; keeps the index valid
    }
  }
  pick = pick < 0 ? 0 : (pick >= N ? N - 1 : pick);
  if (lane == 0) props[l] = pick;
}

template <bool TAB>
__global__ __launch_bounds__(64 * PROPOSE_WAVES) void k_propose(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const double* __restrict__ cpre = RJ.cpre;
  const int64_t nchunks = RJ.nchunks;
  const int b = RJ.b;
  const Unif un = ldc(RJ.un);
  const RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * PROPOSE_WAVES + (threadIdx.x >> 6);
  if (l >= b) return;
  const double T = st->T;
  const double x = stream_uniform(un, 2 * (int64_t)b * st->round + l) * T;
  // first chunk whose inclusive prefix exceeds x
  int64_t lo = 0, hi = nchunks;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (cpre[mid] > x) hi = mid; else lo = mid + 1;
  }
  const int64_t c = (lo < nchunks) ? lo : (int64_t)st->lastpos;
  draw_in_chunk(RJ.u, RJ.N, c, (c > 0) ? cpre[c - 1] : 0.0, x, lane, l, RJ.props);
}

// k_scan_chunks and k_propose in one launch, for up to PS_MAXCH chunks: every
// workgroup forms the inclusive prefix of the chunk sums in its LDS (thread t
// sums a contiguous run of chunks, then the 256 run totals are scanned; the
// same fixed order in every workgroup, so all of them hold the same prefix
// and the same T), and its proposals search it there instead of in global
// memory.  Workgroup 0 records T and the last positive chunk, and the early
// stop (T <= 0) or the exhausted explicit stream as k_scan_chunks does.
constexpr int PS_MAXCH = 4096;

template <bool TAB>
__global__ __launch_bounds__(64 * PROPOSE_WAVES) void k_propose_scan(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const double* __restrict__ csum = RJ.csum;
  const int64_t nch = RJ.nchunks;
  const int b = RJ.b;
  const Unif un = ldc(RJ.un);
  RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  if ((int)blockIdx.x * PROPOSE_WAVES >= b) return;   // uniform: a table's grid fits its largest b
  constexpr int NT = 64 * PROPOSE_WAVES;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t round = st->round;
  if (un.U && 2 * (int64_t)b * (round + 1) > un.nU) {   // uniform
    if (blockIdx.x == 0 && tid == 0) st->status = ST_NOUNIF;
    return;
  }
  __shared__ double pre[PS_MAXCH];
  __shared__ double wsum[PROPOSE_WAVES];
  __shared__ int lsh[PROPOSE_WAVES];
  const int per = (int)((nch + NT - 1) / NT);
  const int cb = tid * per;
  double v = 0.0;
  int lastp = -1;
  for (int i = 0; i < per; ++i) {
    const int c = cb + i;
    if (c < nch) {
      const double x = csum[c];
      v += x;
      pre[c] = v;
      if (x > 0.0) lastp = c;
    }
  }
  const double incl = wave_incl_scan(v);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int t = __shfl_xor(lastp, o, 64);
    lastp = t > lastp ? t : lastp;
  }
  if (lane == 63) wsum[w] = incl;
  if (lane == 0) lsh[w] = lastp;
  double lane_excl = __shfl_up(incl, 1, 64);   // the run totals of the lanes before this one
  if (lane == 0) lane_excl = 0.0;
  __syncthreads();
  double woff = 0.0;
  int lastpos = -1;
#pragma unroll
  for (int q = 0; q < PROPOSE_WAVES; ++q) {
    if (q < w) woff += wsum[q];
    lastpos = lsh[q] > lastpos ? lsh[q] : lastpos;
  }
  const double excl = woff + lane_excl;
  for (int i = 0; i < per; ++i) {
    const int c = cb + i;
    if (c < nch) pre[c] += excl;
  }
  __syncthreads();
  // T is the prefix's last entry, so a draw below T always finds its chunk
  const double T = pre[nch - 1];
  if (!(T > 0.0) || lastpos < 0) {   // uniform
    if (blockIdx.x == 0 && tid == 0) {
      st->T = T;
      st->lastpos = lastpos;
      st->status = ST_EARLY;
    }
    return;
  }
  if (blockIdx.x == 0 && tid == 0) {
    st->T = T;
    st->lastpos = lastpos;
  }
  const int l = blockIdx.x * PROPOSE_WAVES + w;
  if (l >= b) return;
  const double x = stream_uniform(un, 2 * (int64_t)b * round + l) * T;
  int lo = 0, hi = (int)nch;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] > x) hi = mid; else lo = mid + 1;
  }
  const int64_t c = (lo < nch) ? lo : lastpos;
  draw_in_chunk(RJ.u, RJ.N, c, (c > 0) ? pre[c - 1] : 0.0, x, lane, l, RJ.props);
}

// ------------------------------------------------------- gathers at proposals
typedef double rd4 __attribute__((ext_vector_type(4)));

// Fs(i, c) = F(props_i, c) in FP64, row-major with leading dimension ldf
// (and the same rows in FP32 into Fs32 where F is stored in FP32: the product
// term of H reads those, half the bytes, with no rounding);
// ceil(kmax / 256) workgroups per proposal.
template <typename T, bool TAB>
__global__ __launch_bounds__(256) void k_gather_rows(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const T* __restrict__ F = (const T*)RJ.F;
  const int64_t N = RJ.N, ldf = RJ.ldf;
  const int64_t* __restrict__ props = RJ.props;
  double* __restrict__ Fs = RJ.Fs;
  const RoundState* st = RJ.st;
  const int64_t gx = (RJ.kmax + 255) / 256;
  if ((int64_t)blockIdx.x >= gx * RJ.b) return;
  if (st->status != ST_RUNNING) return;
  const int64_t kr = st->k_r;
  const int i = (int)(blockIdx.x / gx);
  const int64_t c = (int64_t)(blockIdx.x % gx) * 256 + threadIdx.x;
  if (c >= kr) return;
  const T v = F[c * N + props[i]];
  Fs[(int64_t)i * ldf + c] = (double)v;
  if constexpr (sizeof(T) == sizeof(float)) RJ.Fs32[(int64_t)i * fs32_ld(ldf) + c] = v;
}

// H = A(S',S') - F(S',:) F(S',:)^T (Alg. 2 step 2), FP64, column-major b x b
// (ld = b), in two launches.  First the product, split along the contraction
// index into partitions of W columns, on the FP64 matrix cores: workgroup
// (x, y, p) with x <= y forms the 16 x 16 tile of rows 16 y .., columns
// 16 x .. of partition p's partial product and writes it and its transpose
// into Hp(p) (workgroups above the diagonal have nothing to do).  Wavefront w
// of eight contracts the 16-column chunks w, w + 8, .. of the partition as
// four 16x16x4 products (lane (g, l16) holds row l16 at column c + 4 g + m of
// product m), so each wavefront's chain of dependent products stays short; the
// eight partial tiles are then added in wavefront order, so the result does
// not depend on scheduling, and a diagonal tile takes every
// entry from its lower half, so each Hp(p), and H, is exactly symmetric.
// The split keeps enough workgroups busy at any k_r.  The cache-line requests
// of the row loads, not the products, set the kernel's pace: where F is
// stored in FP32 (FT = float) the rows come from their FP32 copy, whose
// leading dimension is a multiple of four, so a lane's four columns of a chunk
// are one 16-byte load (FP32 products are exact in FP64).
constexpr int HP_WAVES = 8;
template <bool TAB, typename FT>
__global__ __launch_bounds__(64 * HP_WAVES) void k_gather_Hp(RoundJob jb0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(jb0, tab);
  const int b = RJ.b;
  const FT* __restrict__ Fs;
  if constexpr (sizeof(FT) == sizeof(float)) Fs = RJ.Fs32;
  else Fs = RJ.Fs;
  const int64_t ldf = sizeof(FT) == sizeof(float) ? fs32_ld(RJ.ldf) : RJ.ldf, W = RJ.W;
  double* __restrict__ Hp = RJ.Hp;
  const RoundState* st = RJ.st;
  // workgroup (x, y, z) of an nb x nb x parts grid, folded into blockIdx.x
  const int nb = (b + 15) / 16;
  if ((int64_t)blockIdx.x >= (int64_t)nb * nb * RJ.parts) return;
  const int x = (int)(blockIdx.x % nb), y = (int)((blockIdx.x / nb) % nb), z = (int)(blockIdx.x / (nb * nb));
  if (st->status != ST_RUNNING) return;
  if (x > y) return;
  const int64_t kr = st->k_r;
  const int i0 = 16 * y, j0 = 16 * x;
  const int64_t cbeg = (int64_t)z * W;
  const int64_t cend = (cbeg + W < kr) ? cbeg + W : kr;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const bool ai = i0 + l16 < b, bj = j0 + l16 < b;
  const FT* ar = Fs + (int64_t)(ai ? i0 + l16 : 0) * ldf;
  const FT* br = Fs + (int64_t)(bj ? j0 + l16 : 0) * ldf;
  rd4 acc = {0.0, 0.0, 0.0, 0.0};
  int64_t c = cbeg + 16 * w;
  // four chunks of this wavefront at a time, their loads issued before the products
  constexpr int CS = 16 * HP_WAVES;   // columns per step of all the wavefronts
  for (; c + 3 * CS + 16 <= cend; c += 4 * CS) {
    double av[4][4], bv[4][4];
    if constexpr (sizeof(FT) == sizeof(float)) {
      // c is a multiple of 16 and the row starts 16-byte aligned
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 a4 = *reinterpret_cast<const float4*>(ar + c + CS * u + 4 * g);
        const float4 b4 = *reinterpret_cast<const float4*>(br + c + CS * u + 4 * g);
        av[u][0] = ai ? (double)a4.x : 0.0;
        av[u][1] = ai ? (double)a4.y : 0.0;
        av[u][2] = ai ? (double)a4.z : 0.0;
        av[u][3] = ai ? (double)a4.w : 0.0;
        bv[u][0] = bj ? (double)b4.x : 0.0;
        bv[u][1] = bj ? (double)b4.y : 0.0;
        bv[u][2] = bj ? (double)b4.z : 0.0;
        bv[u][3] = bj ? (double)b4.w : 0.0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          av[u][m] = ai ? (double)ar[c + CS * u + 4 * g + m] : 0.0;
          bv[u][m] = bj ? (double)br[c + CS * u + 4 * g + m] : 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][m], bv[u][m], acc, 0, 0, 0);
  }
  for (; c < cend; c += CS) {
    double av[4], bv[4];
    if (sizeof(FT) == sizeof(float) && c + 16 <= cend) {
      const float4 a4 = *reinterpret_cast<const float4*>(ar + c + 4 * g);
      const float4 b4 = *reinterpret_cast<const float4*>(br + c + 4 * g);
      av[0] = ai ? (double)a4.x : 0.0;
      av[1] = ai ? (double)a4.y : 0.0;
      av[2] = ai ? (double)a4.z : 0.0;
      av[3] = ai ? (double)a4.w : 0.0;
      bv[0] = bj ? (double)b4.x : 0.0;
      bv[1] = bj ? (double)b4.y : 0.0;
      bv[2] = bj ? (double)b4.z : 0.0;
      bv[3] = bj ? (double)b4.w : 0.0;
    } else if (c + 16 <= cend) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        av[m] = ai ? (double)ar[c + 4 * g + m] : 0.0;
        bv[m] = bj ? (double)br[c + 4 * g + m] : 0.0;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t k = c + 4 * g + m;
        av[m] = (ai && k < cend) ? (double)ar[k] : 0.0;
        bv[m] = (bj && k < cend) ? (double)br[k] : 0.0;
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv[m], acc, 0, 0, 0);
  }
  // entry e of lane (g, l16): row 16 y + g + 4 e, column 16 x + l16
  __shared__ double red[HP_WAVES][16][17];
#pragma unroll
  for (int e = 0; e < 4; ++e) red[w][g + 4 * e][l16] = acc[e];
  __syncthreads();
  if (tid >= 256) return;
  const int r = tid >> 4, cc = tid & 15;
  const bool up = x == y && cc > r;
  const int rr = up ? cc : r, ck = up ? r : cc;
  double v = red[0][rr][ck];
#pragma unroll
  for (int q = 1; q < HP_WAVES; ++q) v += red[q][rr][ck];
  const int i = i0 + r, j = j0 + cc;
  if (i < b && j < b) {
    double* hp = Hp + (int64_t)z * b * b;
    hp[(int64_t)j * b + i] = v;
    hp[(int64_t)i * b + j] = v;
  }
}

// Second launch: H(i, j) = kappa(x_i, x_j) - sum over the partitions, in
// partition order.
template <bool TAB>
__global__ __launch_bounds__(256) void k_gather_Hs(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const double* __restrict__ X = RJ.X;
  const int d = RJ.d, b = RJ.b, parts = RJ.parts;
  const KParams kp = ldc(RJ.kp);
  const int64_t* __restrict__ props = RJ.props;
  const double* __restrict__ Hp = RJ.Hp;
  double* __restrict__ H = RJ.H;
  const RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (int64_t)b * b) return;
  const int i = (int)(q % b), j = (int)(q / b);
  double acc = 0.0;
  for (int p = 0; p < parts; ++p) acc += Hp[(int64_t)p * b * b + q];
  const double* xi = X + props[i] * d;
  const double* xj = X + props[j] * d;
  H[q] = kappa_r2(sqdist(xi, xj, d), kp) - acc;
}

// The same for large d, one 16 x 16 block of H per workgroup: the coordinates
// of its 16 + 16 proposals are staged through LDS 64 dims at a time (each row
// is read from L2 once per block instead of once per entry); every entry sums
// its squared differences in the same order as sqdist.
constexpr int HS_T = 16, HS_DC = 64;
template <bool TAB>
__global__ __launch_bounds__(256) void k_gather_Hs_tiled(RoundJob jb0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(jb0, tab);
  const double* __restrict__ X = RJ.X;
  const int d = RJ.d, b = RJ.b, parts = RJ.parts;
  const KParams kp = ldc(RJ.kp);
  const int64_t* __restrict__ props = RJ.props;
  const double* __restrict__ Hp = RJ.Hp;
  double* __restrict__ H = RJ.H;
  const RoundState* st = RJ.st;
  // block (bx, by) of the ceil(b / 16)^2 blocks, folded into blockIdx.x
  const int nbt = (b + HS_T - 1) / HS_T;
  if ((int)blockIdx.x >= nbt * nbt) return;
  if (st->status != ST_RUNNING) return;
  __shared__ double xs[2][HS_T][HS_DC + 1];   // [0]: rows i of the block, [1]: rows j
  const int tid = threadIdx.x, ti = tid % HS_T, tj = tid / HS_T;
  const int i0 = ((int)blockIdx.x % nbt) * HS_T, j0 = ((int)blockIdx.x / nbt) * HS_T;
  // blocks above the diagonal: their entries are written by the block below
  // it (the same sums and the same partial products, so H stays exactly
  // symmetric)
  if (j0 > i0) return;
  const int i = i0 + ti, j = j0 + tj;
  // staging: thread tid copies dims (tid % 64) of rows (tid / 64) + 4 m, m < 8, of the 32 rows
  const int sd = tid % HS_DC, sr = tid / HS_DC;
  const double* src[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int r = sr + 4 * m;                       // 0..31: rows i0.. (r < 16), then j0..
    const int li = r < HS_T ? i0 + r : j0 + r - HS_T;
    src[m] = X + props[li < b ? li : b - 1] * d;
  }
  // the partial products, summed in partition order, loaded beside the first
  // chunk's coordinates
  const bool in = i < b && j < b;
  const int64_t q = (int64_t)j * b + i;
  double acc = 0.0;
  if (in)
    for (int p = 0; p < parts; ++p) acc += Hp[(int64_t)p * b * b + q];
  double sum = 0.0;
  // each chunk's coordinates are loaded into registers one chunk ahead, so
  // their loads overlap the previous chunk's sums
  double nx[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) nx[m] = sd < d ? src[m][sd] : 0.0;
  for (int k0 = 0; k0 < d; k0 += HS_DC) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int r = sr + 4 * m;
      xs[r / HS_T][r % HS_T][sd] = nx[m];
    }
    __syncthreads();
    if (k0 + HS_DC < d) {
#pragma unroll
      for (int m = 0; m < 8; ++m) nx[m] = k0 + HS_DC + sd < d ? src[m][k0 + HS_DC + sd] : 0.0;
    }
    const int ke = d - k0 < HS_DC ? d - k0 : HS_DC;
    for (int t = 0; t < ke; ++t) {
      const double e = xs[0][ti][t] - xs[1][tj][t];
      sum += e * e;
    }
  }
  if (in) {
    const double h = kappa_r2(sum, kp) - acc;
    H[q] = h;
    if (j0 < i0) H[(int64_t)i * b + j] = h;
  }
}

// ------------------------------------------------- RejectionSampleSubmatrix
// Alg. 1 on the b x b residual submatrix, in one workgroup, right-looking and
// in place: accepted column i is scaled by 1/sqrt(h_ii) and the trailing
// lower triangle receives the rank-one Schur update.  Storage: matrix-core
// tiles in registers (b <= 256, below) or the full column-major matrix in
// global memory.
// Rules beyond the printed test u_i * V < h_ii: a proposal equal to one
// already accepted in this round is rejected, and at most k - k_r proposals are
// accepted.  keep_all runs block RPCholesky (Alg. 7) instead: every test takes
// V = 0, so each distinct proposal with a positive residual is kept.
// Outputs: accepted local indices, the new pivots, u = 0 at the new pivots,
// and the lower Cholesky factor L of H(T,T) left in H: the scaled
// column of accepted proposal i is column i of H (rows at and below i), so
// L(a, c) = H(acc[a], acc[c]) (read through LFactor).
struct FullGlobal {
  double* p;
  int b;
  __device__ inline double& at(int j, int i) const { return p[(int64_t)i * b + j]; }
};

template <class Store>
__device__ void reject_body(Store S, int b, const int64_t* __restrict__ props, Unif un,
                            RoundState* st, int32_t* __restrict__ acc_out,
                            int64_t* __restrict__ pivots, double* __restrict__ u, int64_t kmax,
                            int keep_all, unsigned char* tk, int* dec, short* accl, double* sqv) {
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, w = tid >> 6, nw = nthr >> 6;
  const int64_t kr = st->k_r;
  const int64_t round = st->round;
  const int cap = (int)((kmax - kr) < b ? (kmax - kr) : b);
  double uloc = 0.0, V = 0.0;
  int prev = -1;
  if (tid < b) {
    uloc = S.at(tid, tid);
    V = keep_all ? 0.0 : stream_uniform(un, 2 * (int64_t)b * round + b + tid);
    const int64_t me = props[tid];
    for (int q = tid - 1; q >= 0; --q)
      if (props[q] == me) { prev = q; break; }
    tk[tid] = 0;
  }
  __syncthreads();
  int nacc = 0;
  for (int i = 0; i < b && nacc < cap; ++i) {
    if (tid == i) {
      const double h = S.at(i, i);
      const bool dup = prev >= 0 && tk[prev];
      const bool a = !dup && (uloc * V < h);
      tk[i] = (a || dup) ? 1 : 0;
      dec[i & 1] = a ? 1 : 0;
      if (a) {
        accl[nacc] = (short)i;
        sqv[i & 1] = sqrt(h);   // every thread scales by this; H(i, i) itself is rewritten below
      }
    }
    __syncthreads();
    if (!dec[i & 1]) continue;
    const double sq = sqv[i & 1];
    for (int j = i + tid; j < b; j += nthr) S.at(j, i) = S.at(j, i) / sq;
    __syncthreads();
    for (int l = i + 1 + w; l < b; l += nw) {
      const double Ll = S.at(l, i);
      for (int j = l + lane; j < b; j += 64) S.at(j, l) -= S.at(j, i) * Ll;
    }
    __syncthreads();
    ++nacc;
  }
  __syncthreads();
  // L(T,T) stays in H: entry (a, c) is S.at(accl[a], accl[c]) (see LFactor)
  for (int a = tid; a < nacc; a += nthr) {
    const int64_t p = props[accl[a]];
    acc_out[a] = accl[a];
    pivots[kr + a] = p;
    u[p] = 0.0;
  }
  if (tid == 0) st->s_r = nacc;
}

// Tiled form for b <= 256, one workgroup of eight wavefronts.  Wavefront 0
// runs the tests; the other seven hold the trailing submatrix as 16 x 16
// tiles in FP64 matrix-core accumulators.  The tiles of the lower triangle
// are numbered down the block columns, t = T0(L) + J - L for tile (J, L),
// J >= L, T0(L) = L nbk - L (L - 1) / 2, and tile t belongs to tile wavefront
// t mod 7 (its slot t / 7), so the tiles of block columns L >= I are a range
// of each wavefront's slots.  Entry i of lane (g, n) of a tile is row
// 16 J + g + 4 i, column 16 L + n: the layout of the FP64 16x16x4 product's
// accumulator.  The proposals are taken 16 at a time (block column I):
//  1. wavefront 0 runs the tests of Alg. 1 on the diagonal block and forms
//     the block's columns of the factor and the inverse X of their factor;
//  2. the panel below the block is solved against the accepted columns as a
//     product with X, four matrix-core products per tile;
//  3. the trailing tiles receive the rank-16 update on the matrix cores, four
//     products per tile (rejected columns are zero).
// The register-resident form defers 2 and 3 of block I - 1 into block I
// (look-ahead): before block I's tests only the panel row P_I and the
// diagonal tile (I, I) are computed (by that tile's owner); the rest of the
// panel runs beside the first half of the tests and the rest of the update
// beside the second half (X double-buffered, barriers on LDS only).  The
// block-column buffer is double-buffered so a block's copy does not
// overwrite the previous panel while it is still being applied.  Block 0's
// diagonal block is read from H itself, so its tests start while the tile
// wavefronts are still loading.
// For 256 < b <= 512 the triangle (up to 528 tiles, 1 MiB) does not fit the
// register file; the GT form keeps the trailing tiles in H and streams them
// through the steps (three full barriers per block; there the trailing
// update, not the tests, sets the pace, so the look-ahead gains nothing).
// Duplicates: the latest earlier proposal of the same point is found through
// chained hash buckets in LDS (the chains are short; each is walked in full,
// so the answer does not depend on the order of the insertions).
constexpr int RT = 16;                  // tile edge
constexpr int REJECT_T_THREADS = 512;
constexpr int REJECT_T_BMAX = 256;
constexpr int REJECT_G_BMAX = REJECT_TILED_BMAX;   // the form with the trailing tiles in global memory
constexpr int REJECT_T_TW = 7;          // tile wavefronts
constexpr int REJECT_T_TPW = 20;        // tiles per tile wavefront: 136 / 7, rounded up
constexpr int QS = 18;                  // LDS row stride (doubles) of the block-column buffer
constexpr int GT_RC = 13;               // b > 256: block columns whose tiles stay in registers
constexpr int GT_TPW = 13;              // their tiles per tile wavefront: 91 / 7
constexpr int DUP_HBITS = 12;           // 4096 hash buckets

// LDS of the tiled form.  The small arrays come first, at addresses that fit
// the offset field of the LDS instructions.
template <int BM>
struct RejectLds {
  double BC[RT][RT];       // BC[ii][r]: column ii of the diagonal block (unscaled) when its test runs
  double XB[2][RT * RT];   // X of the last two blocks, X(r, c) at [r * RT + c]
  double rsq[RT];          // 1/sqrt(h) of the block's accepted proposals (0: rejected)
  double uv[BM];           // u_i V_i of the test
  short prv[BM], accl[BM];
  unsigned char tk[BM];
  int bmask;
  alignas(16) double Q[2][BM][QS];   // block columns
};
// The duplicate search's scratch, in the block-column buffer before the first block.
struct DupScratch {
  int64_t pr[REJECT_G_BMAX];
  int nxt[REJECT_G_BMAX];
  int head[1 << DUP_HBITS];
};
static_assert(sizeof(DupScratch) <= sizeof(double) * 2 * REJECT_T_BMAX * QS, "duplicate scratch exceeds the block buffer");

__device__ __forceinline__ int dup_bucket(int64_t p) {
  return (int)(((uint64_t)p * 0x9E3779B97F4A7C15ull) >> (64 - DUP_HBITS));
}

// Workgroup barrier for LDS traffic only (it does not wait for global stores
// in flight): the tiled forms exchange data between their waves only through
// LDS (the factor columns stored to H are read by later kernels, and every
// tile load from a column block of H has been consumed before that block's
// columns are written).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool GT, bool TAB>
__global__ __launch_bounds__(REJECT_T_THREADS) void k_reject_tiled(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  double* __restrict__ H = RJ.H;
  const int b = RJ.b;
  const int64_t* __restrict__ props = RJ.props;
  const Unif un = ldc(RJ.un);
  RoundState* st = RJ.st;
  int32_t* __restrict__ acc_out = RJ.acc;
  int64_t* __restrict__ pivots = RJ.pivots;
  double* __restrict__ u = RJ.u;
  const int64_t kmax = RJ.kmax;
  const int keep_all = RJ.keep_all;
  if (st->status != ST_RUNNING) return;
  constexpr int BM = GT ? REJECT_G_BMAX : REJECT_T_BMAX;
  constexpr bool LA = !GT;
  __shared__ RejectLds<BM> sm;
  DupScratch& dsc = *reinterpret_cast<DupScratch*>(&sm.Q[0][0][0]);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: tile coordinates stay scalar
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t kr = st->k_r, round = st->round;
  const int cap = (int)((kmax - kr) < b ? (kmax - kr) : b);
  const int nbk = (b + RT - 1) / RT;
  const int ntile = nbk * (nbk + 1) / 2;

  int nacc = 0;
  if (w == 0) {
    // ---- per-proposal state (proposals lane, lane + 64, ...) and the
    // duplicate chains.  This wavefront's loads are issued before the start
    // barrier (P), the tile wavefronts' tile loads after it, so these do not
    // queue behind them.
    constexpr int PW = BM / 64;
    // block 0's diagonal block, row l16 (no update is pending there), kept in
    // rows 0..15 of the second block buffer, which no block column reaches
    double dr0[RT], hv[PW], uu[PW];
    int64_t pv[PW];
#pragma unroll
    for (int c = 0; c < RT; ++c) dr0[c] = (l16 < b && c < b) ? H[(int64_t)c * b + l16] : 0.0;
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int i = lane + 64 * q;
      pv[q] = i < b ? props[i] : 0;
      hv[q] = i < b ? H[(int64_t)i * b + i] : 0.0;
      uu[q] = (i < b && un.U) ? un.U[2 * (int64_t)b * round + b + i] : 0.0;
    }
    lds_sync();   // (P)
    for (int q = lane; q < (1 << DUP_HBITS) / 4; q += 64)
      reinterpret_cast<int4*>(dsc.head)[q] = make_int4(-1, -1, -1, -1);
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int i = lane + 64 * q;
      if (i < b) {
        sm.tk[i] = 0;
        dsc.pr[i] = pv[q];
        dsc.nxt[i] = atomicExch(&dsc.head[dup_bucket(pv[q])], i);
      }
    }
    for (int i = lane; i < b; i += 64) {
      const int64_t p = dsc.pr[i];
      int best = -1;
      int q = dsc.head[dup_bucket(p)];
      for (int n = 0; q >= 0 && n < b; ++n) {   // a chain holds each proposal once
        if (q < i && q > best && dsc.pr[q] == p) best = q;
        q = dsc.nxt[q];
      }
      sm.prv[i] = (short)best;
    }
    if (LA && g == 0)
#pragma unroll
      for (int c = 0; c < RT; ++c) sm.Q[1][l16][c] = dr0[c];
    lds_sync();   // (0) the scratch is free for the block columns; the uniforms are in uv
    // u_i V_i of the tests (keep_all: V = 0)
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      const int i = lane + 64 * q;
      if (i < b) sm.uv[i] = keep_all ? 0.0 : hv[q] * (un.U ? uu[q] : sm.uv[i]);
    }

    // ---- the tests.  Lane r (mod 16) keeps row 16 I + r of the (symmetric)
    // diagonal block.  The update after an accepted proposal ii is written as
    // T(r, c) -= (T(r, ii) / h) T(c, ii), the same rank-one update as with the
    // scaled column, so the chain from one test to the next holds a
    // reciprocal but no square root; the scaled columns, 1/sqrt(h) and the
    // outputs are formed for the whole block afterwards.  Straight-line code:
    // a rejected proposal has a zero multiplier.  Column ii is written to BC
    // at the start of its step (the row of the next test by readlane, the
    // rest through LDS, needed no earlier than the test after next); BC then
    // holds every unscaled column of the block's factor.
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      if (!LA || I > 0) {
        if constexpr (LA) lds_sync();       // (1) the diagonal block of block column I is in LDS
        else __syncthreads();                // (1) block column I is in LDS
      }
      const double* src = (LA && I == 0) ? &sm.Q[1][l16][0] : &sm.Q[I & 1][RT * I + l16][0];
      double dr[RT];
#pragma unroll
      for (int c = 0; c < RT; ++c) dr[c] = src[c];
      const int iL = RT * I + l16;
      double uvL = 0.0;
      int pL = -1;
      bool dupL = false;
      if (iL < b) {
        uvL = sm.uv[iL];
        const int p = sm.prv[iL];
        if (p >= RT * I) pL = p - RT * I;
        else if (p >= 0) dupL = sm.tk[p] != 0;
      }
      const unsigned dup_before = (unsigned)__ballot(dupL) & 0xffffu;
      const int bl = b - RT * I;
      const unsigned okm = bl >= RT ? 0xffffu : ((1u << bl) - 1u);
      const int capL = cap - nacc;
      unsigned mask = 0, taken = 0;
      int cnt = 0;
      // column ii goes to BC, and its entries below the next row are read
      // back, at the end of step ii - 1, so that the LDS round trip overlaps
      // the next test
      double bcn[RT];
      sm.BC[0][l16] = dr[0];
#pragma unroll
      for (int c = 2; c < RT; ++c) bcn[c] = sm.BC[0][c];
#pragma unroll
      for (int ii = 0; ii < RT; ++ii) {
        if constexpr (LA) {
          if (ii == RT / 2) lds_sync();   // (m) the panel of the previous block is complete
        }
        const double bn = readlane_f64(dr[ii], ii + 1 < RT ? ii + 1 : ii);
        double bc[RT];
#pragma unroll
        for (int c = ii + 2; c < RT; ++c) bc[c] = bcn[c];
        // the test of proposal 16 I + ii, from lane ii's values: its u V
        // against h = its diagonal entry, and whether an earlier proposal of
        // the same point was taken (before this block: dup_before; in it:
        // the taken mask at its local index)
        // 1/h: hardware reciprocal and two Newton steps (exact for h = 1),
        // formed beside the decision; where the proposal is not accepted
        // (h may then be zero or negative) the multiplier is selected away
        const double h = readlane_f64(dr[ii], ii);
        double inv = __builtin_amdgcn_rcp(h);
        inv = fma(inv, fma(-h, inv, 1.0), inv);
        inv = fma(inv, fma(-h, inv, 1.0), inv);
        const double tv = dr[ii] * inv;
        const unsigned long long lt = __ballot(uvL < dr[ii]);
        const int pq = __builtin_amdgcn_readlane(pL, ii);
        const unsigned dup = ((dup_before >> ii) | ((taken >> (pq & 15)) & (unsigned)(pq >= 0))) & 1u;
        const unsigned below_cap = (unsigned)(cnt - capL) >> 31;
        const unsigned av = ~dup & (unsigned)(lt >> ii) & (okm >> ii) & below_cap & 1u;
        taken |= (av | dup) << ii;
        mask |= av << ii;
        cnt += (int)av;
        const double t = av ? tv : 0.0;
        if (ii + 1 < RT) {
          dr[ii + 1] = fma(-t, bn, dr[ii + 1]);
          sm.BC[ii + 1][l16] = dr[ii + 1];
        }
#pragma unroll
        for (int c = ii + 2; c < RT; ++c) dr[c] = fma(-t, bc[c], dr[c]);
#pragma unroll
        for (int c = ii + 3; c < RT; ++c) bcn[c] = sm.BC[ii + 1][c];
      }
      // ---- the block's outputs.  Lane c forms 1/sqrt(h_c) from its diagonal
      // entry BC[c][c]; column ii of the factor (zero for a rejected
      // proposal) is BC[ii][r] / sqrt(h_ii), rows r >= ii, stored to column
      // 16 I + ii of H by lanes (g, r) for ii = g, g + 4, g + 8, g + 12.
      {
        const double hL = sm.BC[l16][l16];
        const double rsL = ((mask >> l16) & 1u) ? 1.0 / sqrt(hL) : 0.0;
        if (lane < RT) {
          sm.rsq[lane] = rsL;
          if (iL < b) sm.tk[iL] = (taken >> lane) & 1u;
          if ((mask >> lane) & 1u) sm.accl[nacc + __popc(mask & ((1u << lane) - 1u))] = (short)iL;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ii = g + 4 * i;
          if (l16 >= ii && iL < b && RT * I + ii < b)
            H[(int64_t)(RT * I + ii) * b + iL] = sm.BC[ii][l16] * sm.rsq[ii];
        }
      }
      // X = L^{-1} restricted to the accepted proposals (rejected rows and
      // columns come out zero): lane c forms column c by forward
      // substitution on the unscaled columns, L(r, k) = BC[k][r] rs_k:
      // x_k = y_k rs_k, then y_r -= BC[k][r] (x_k rs_k) for r > k
      {
        double y[RT];
        // the right-hand side e_c, from a value of this block (a
        // loop-invariant one would be hoisted out of the block loop and held
        // in registers through it)
        const double one = (double)(mask | 1u) / (double)(mask | 1u);
#pragma unroll
        for (int r = 0; r < RT; ++r) y[r] = (r == l16) ? one : 0.0;
#pragma unroll
        for (int k = 0; k < RT; ++k) {
          const double rk = sm.rsq[k];
          const double xk = y[k] * rk;
          const double zk = xk * rk;
          y[k] = xk;
#pragma unroll
          for (int r = k + 1; r < RT; ++r) y[r] = fma(-sm.BC[k][r], zk, y[r]);
        }
        double* xo = sm.XB[I & 1];
        if (lane < RT)
#pragma unroll
          for (int r = 0; r < RT; ++r) xo[r * RT + lane] = y[r];
      }
      // X's strictly lower part into the upper triangle of the block's
      // diagonal block of H, no longer read here (the inverse-factor kernels
      // solve by blocks with it; see linv_blocks): lane (g, c) stores rows
      // g, g + 4, g + 8, g + 12 of column c, read back from LDS
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = g + 4 * i;
        if (r > l16 && RT * I + r < b)
          H[(int64_t)(RT * I + r) * b + RT * I + l16] = sm.XB[I & 1][r * RT + l16];
      }
      if (lane == 0) sm.bmask = (int)mask;
      if constexpr (LA) {
        lds_sync();   // (2) decisions, rsq and X are in LDS
        if (mask == 0) continue;
      } else {
        __syncthreads();   // (2) decisions, rsq and X are in LDS
        if (mask == 0) continue;
        __syncthreads();   // (3) the panel is solved
      }
      nacc += __popc(mask);
    }
  } else if constexpr (!GT) {
    const int wt = w - 1;
    const int nslot = ntile > wt ? (ntile - wt + REJECT_T_TW - 1) / REJECT_T_TW : 0;
    rd4 tr[REJECT_T_TPW];
    // (J, L) of this wavefront's slots, four bits each, four slots per word
    // (scalar registers); slots past the last tile name tile (0, 0)
    unsigned pk[(REJECT_T_TPW + 3) / 4];
    {
#pragma unroll
      for (int q = 0; q < (REJECT_T_TPW + 3) / 4; ++q) pk[q] = 0;
      int L = 0, off = wt;   // tile wt + 7 k: (L + off, L)
#pragma unroll
      for (int k = 0; k < REJECT_T_TPW; ++k) {
        while (L < nbk && off >= nbk - L) {
          off -= nbk - L;
          ++L;
        }
        if (k < nslot) pk[k / 4] |= (unsigned)(((L + off) & 15) | ((L & 15) << 4)) << (8 * (k % 4));
        off += REJECT_T_TW;
      }
    }
    // f(k, J, L) for the slots k in [lo, hi), lo <= hi (a bit mask of the
    // range: a comparison with a single slot index would let the compiler
    // index the tile registers dynamically, which puts them in scratch)
    auto for_slots = [&](int lo, int hi, auto f) __attribute__((always_inline)) {
      const unsigned sel = ((1u << hi) - 1u) ^ ((1u << lo) - 1u);
#pragma unroll
      for (int k = 0; k < REJECT_T_TPW; ++k) {
        if ((sel >> k) & 1u) {
          const unsigned e = pk[k / 4] >> (8 * (k % 4));
          f(k, (int)(e & 15), (int)((e >> 4) & 15));
        }
      }
    };
    // this wavefront's tiles of H (zero padding), read along rows of the
    // symmetric H so that a load instruction covers four 128-byte runs; the
    // loads are unconditional (clamped indices) so that all stay in flight
    lds_sync();   // (P)
#pragma unroll
    for (int k = 0; k < REJECT_T_TPW; ++k) {
      const unsigned e = pk[k / 4] >> (8 * (k % 4));
      const int J = (int)(e & 15), L = (int)((e >> 4) & 15);
      const int col = RT * L + l16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = RT * J + g + 4 * i;
        tr[k][i] = H[(int64_t)(row < b ? row : b - 1) * b + (col < b ? col : b - 1)];
      }
    }
    // the counter-based uniforms V_i of the tests, while the loads are in flight
    if (!keep_all && !un.U)
      for (int i = tid - 64; i < b; i += REJECT_T_THREADS - 64)
        sm.uv[i] = philox_uniform(un.seed, (uint64_t)(2 * (int64_t)b * round + b + i));
    lds_sync();   // (0)
    // zero padding (after (0): block 0's tests need no tile, so they start
    // while these loads are in flight)
    for_slots(0, nslot, [&](int k, int J, int L) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (RT * J + g + 4 * i >= b || RT * L + l16 >= b) tr[k][i] = 0.0;
    });
    // T(J, L) -= P_J P_L^T for the slots in [lo, hi), four k-steps of four
    // columns (rejected columns of P are zero), P the previous block's solved
    // panel; a tile's eight operands are read before its products
    auto update = [&](double(*P)[QS], int lo, int hi) __attribute__((always_inline)) {
      for_slots(lo, hi, [&](int k, int J, int L) {
        double av[4], bv[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          av[ks] = P[RT * J + l16][4 * ks + g];
          bv[ks] = P[RT * L + l16][4 * ks + g];
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) tr[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[ks], bv[ks], tr[k], 0, 0, 0);
      });
    };
    // the slots in [lo, hi) into the rows of their block J of the buffer
    auto copy_to = [&](double(*Qd)[QS], int lo, int hi) __attribute__((always_inline)) {
      for_slots(lo, hi, [&](int k, int J, int L) {
#pragma unroll
        for (int i = 0; i < 4; ++i) Qd[RT * J + g + 4 * i][l16] = tr[k][i];
      });
    };
    // panel rows J >= Jlo of block Ip (spread: row J to tile wavefront
    // (J - Jlo) mod 7; else row Jlo only, by the caller): P_J = Q_J X^T from
    // the copy of block column Ip, in place, and the accepted columns into H
    auto panel = [&](double(*Qs)[QS], const double* X, int Ip, int Jlo, bool spread) __attribute__((always_inline)) {
      const int jb = spread ? Jlo + wt : Jlo, je = spread ? nbk : Jlo + 1;
      for (int J = jb; J < je; J += REJECT_T_TW) {
        double av[4], xv[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          av[ks] = Qs[RT * J + l16][4 * ks + g];
          xv[ks] = X[l16 * RT + 4 * ks + g];
        }
        rd4 pj = rd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) pj = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], xv[ks], pj, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) Qs[RT * J + g + 4 * i][l16] = pj[i];
        if (RT * Ip + l16 < b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = RT * J + g + 4 * i;
            if (row < b) H[(int64_t)(RT * Ip + l16) * b + row] = pj[i];
          }
      }
    };
    // Look-ahead: the panel and the rank-16 update of block I - 1 run during
    // block I.  Before the tests of block I only the panel row P_I and the
    // diagonal tile (I, I) are computed, by that tile's owner (the first
    // tile of block column I); the rest of the panel runs beside the first
    // half of the tests and the rest of the update beside the second half,
    // the block's outputs and its inverse factor (wavefront 0 takes the
    // barrier (m) between them inside its test loop).
    int pmask = 0;   // accepted columns of the previous block (panel and update pending)
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      double(*Qb)[QS] = sm.Q[I & 1];
      double(*Qp)[QS] = sm.Q[(I + 1) & 1];         // block column I - 1, becoming its panel
      const double* Xp = sm.XB[(I + 1) & 1];       // X of block I - 1
      // slots of block columns >= I start at k0, those of block column I end
      // before k2; the diagonal tile (I, I) is tile T0(I)
      const int T0 = I * nbk - I * (I - 1) / 2, T1 = T0 + nbk - I;
      const int k0 = T0 > wt ? (T0 - wt + REJECT_T_TW - 1) / REJECT_T_TW : 0;
      const int k2 = T1 > wt ? (T1 - wt + REJECT_T_TW - 1) / REJECT_T_TW : 0;
      const bool own = T0 % REJECT_T_TW == wt;
      const int k1 = own ? k0 + 1 : k0;
      if (I > 0) {
        if (own) {
          // panel row I of block I - 1 and the diagonal tile's update with
          // it (this wavefront's own LDS writes are ordered before its
          // reads); the other waves read P_I only after (m)
          if (pmask) panel(Qp, Xp, I - 1, I, false);
          // update and copy in one pass over the slot (two separate
          // conditional passes over the same tile spill the tile registers)
          for_slots(k0, k0 + 1, [&](int k, int J, int L) {
            if (pmask) {
              double av[4];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) av[ks] = Qp[RT * I + l16][4 * ks + g];
#pragma unroll
              for (int ks = 0; ks < 4; ++ks) tr[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[ks], av[ks], tr[k], 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) Qb[RT * I + g + 4 * i][l16] = tr[k][i];
          });
        }
        lds_sync();   // (1)
      }
      if (pmask) panel(Qp, Xp, I - 1, I + 1, true);
      lds_sync();   // (m)
      if (pmask) update(Qp, k1, nslot);
      copy_to(Qb, k1, k2);
      lds_sync();   // (2)
      const int mask = sm.bmask;
      pmask = mask;
      if (mask == 0) continue;
      nacc += __popc(mask);
    }
  } else {
    // 256 < b <= 512: the trailing triangle (up to 528 tiles, 1 MiB) does
    // not fit the register file.  The tiles of the last GT_RC block columns
    // (L >= L0) are held in registers as in the form above (numbered down
    // those columns, tile t of that sub-triangle to tile wavefront t mod 7).
    // The tiles of the earlier block columns stay in H itself: tile (J, L),
    // J >= L, element (r, c) (row 16 J + r, column 16 L + c of the residual)
    // at H[(16 J + r) b + 16 L + c], the upper triangle of the column-major H
    // for J > L and the whole diagonal block for J = L (the factor goes to the
    // lower triangle of block columns already consumed, so the two never
    // overlap); each of their updates is a load, four matrix-core products
    // and a store, out of the XCD's L2.  Per block I: 1. block column I with
    // the pending update (of block I - 1) to LDS; 2. the rest of the pending
    // update, beside the tests; 3. the panel below the block.
    const int wt = w - 1;
    const int L0 = nbk > GT_RC ? nbk - GT_RC : 0;   // first register-resident block column
    const int mr = nbk - L0;
    const int ntr = mr * (mr + 1) / 2;
    const int nslot = ntr > wt ? (ntr - wt + REJECT_T_TW - 1) / REJECT_T_TW : 0;
    // first tile of sub-triangle column L (L0 <= L <= nbk), and this
    // wavefront's first slot at or after sub-triangle tile T
    auto t0r = [&](int L) __attribute__((always_inline)) {
      const int q = L - L0;
      return q * mr - q * (q - 1) / 2;
    };
    auto kfirst = [&](int T) __attribute__((always_inline)) {
      return T > wt ? (T - wt + REJECT_T_TW - 1) / REJECT_T_TW : 0;
    };
    rd4 tr[GT_TPW];
    // (J, L) of this wavefront's slots, eight bits each, two slots per word
    // (scalar registers); slots past the last tile name tile (0, 0)
    unsigned pk[(GT_TPW + 1) / 2];
    {
#pragma unroll
      for (int q = 0; q < (GT_TPW + 1) / 2; ++q) pk[q] = 0;
      int L = L0, off = wt;   // tile wt + 7 k of the sub-triangle: (L + off, L)
#pragma unroll
      for (int k = 0; k < GT_TPW; ++k) {
        while (L < nbk && off >= nbk - L) {
          off -= nbk - L;
          ++L;
        }
        if (k < nslot) pk[k / 2] |= (unsigned)(((L + off) & 255) | ((L & 255) << 8)) << (16 * (k % 2));
        off += REJECT_T_TW;
      }
    }
    // f(k, J, L) for the slots k in [lo, hi), lo <= hi (a bit mask, as above)
    auto for_slots = [&](int lo, int hi, auto f) __attribute__((always_inline)) {
      const unsigned sel = ((1u << hi) - 1u) ^ ((1u << lo) - 1u);
#pragma unroll
      for (int k = 0; k < GT_TPW; ++k) {
        if ((sel >> k) & 1u) {
          const unsigned e = pk[k / 2] >> (16 * (k % 2));
          f(k, (int)(e & 255), (int)((e >> 8) & 255));
        }
      }
    };
    // tile (J, L) from H (indices clamped into the matrix; see tpad)
    auto tload = [&](int J, int L) __attribute__((always_inline)) {
      rd4 t;
      const int col = RT * L + l16;
      const int cc = col < b ? col : b - 1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = RT * J + g + 4 * i;
        t[i] = H[(int64_t)(row < b ? row : b - 1) * b + cc];
      }
      return t;
    };
    // zero padding outside the b x b matrix
    auto tpad = [&](rd4& t, int J, int L) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (RT * J + g + 4 * i >= b || RT * L + l16 >= b) t[i] = 0.0;
    };
    auto tstore = [&](const rd4& t, int J, int L) __attribute__((always_inline)) {
      const int col = RT * L + l16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = RT * J + g + 4 * i;
        if (row < b && col < b) H[(int64_t)row * b + col] = t[i];
      }
    };
    // T(J, L) -= P_J P_L^T, P the previous block's solved panel
    auto tupd = [&](rd4 t, double(*P)[QS], int J, int L) __attribute__((always_inline)) {
      double av[4], bv[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        av[ks] = P[RT * J + l16][4 * ks + g];
        bv[ks] = P[RT * L + l16][4 * ks + g];
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) t = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[ks], bv[ks], t, 0, 0, 0);
      return t;
    };
    constexpr int NB1 = (REJECT_G_BMAX / RT + REJECT_T_TW - 1) / REJECT_T_TW;   // tiles of a block column per wavefront
    constexpr int NB = 4;   // tiles of H in flight in the update (the register tiles leave room for four)
    lds_sync();   // (P)
    // the register-resident tiles, all loads in flight (clamped indices)
#pragma unroll
    for (int k = 0; k < GT_TPW; ++k) {
      const unsigned e = pk[k / 2] >> (16 * (k % 2));
      tr[k] = tload((int)(e & 255), (int)((e >> 8) & 255));
    }
    if (!keep_all && !un.U)
      for (int i = tid - 64; i < b; i += REJECT_T_THREADS - 64)
        sm.uv[i] = philox_uniform(un.seed, (uint64_t)(2 * (int64_t)b * round + b + i));
    lds_sync();   // (0)
    for_slots(0, nslot, [&](int k, int J, int L) { tpad(tr[k], J, L); });
    int pmask = 0;
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      double(*Qb)[QS] = sm.Q[I & 1];
      double(*Qp)[QS] = sm.Q[(I + 1) & 1];
      // 1. block column I (tiles (J, I), J >= I) with the pending update, to LDS
      if (I < L0) {
        rd4 t[NB1];
#pragma unroll
        for (int n = 0; n < NB1; ++n) {
          const int J = I + wt + REJECT_T_TW * n;
          t[n] = tload(J < nbk ? J : nbk - 1, I);
        }
#pragma unroll
        for (int n = 0; n < NB1; ++n) {
          const int J = I + wt + REJECT_T_TW * n;
          if (J < nbk) {
            tpad(t[n], J, I);
            if (pmask) t[n] = tupd(t[n], Qp, J, I);
#pragma unroll
            for (int i = 0; i < 4; ++i) Qb[RT * J + g + 4 * i][l16] = t[n][i];
          }
        }
      } else {
        // register tiles of block column I: update and copy in one pass
        for_slots(kfirst(t0r(I)), kfirst(t0r(I + 1)), [&](int k, int J, int L) {
          if (pmask) tr[k] = tupd(tr[k], Qp, J, L);
#pragma unroll
          for (int i = 0; i < 4; ++i) Qb[RT * J + g + 4 * i][l16] = tr[k][i];
        });
      }
      __syncthreads();   // (1)
      // 2. the rest of the pending update, beside the tests
      if (pmask) {
        // tiles in H: (J, L), I < L < L0, numbered down the block columns,
        // tile q to tile wavefront q mod 7, NB loads in flight
        if (I + 1 < L0) {
          const int m = (L0 - I - 1) * nbk - ((L0 - 1) * L0 / 2 - I * (I + 1) / 2);
          int L = I + 1, off = wt;   // tile q: (L + off, L)
          for (int q = wt; q < m; q += REJECT_T_TW * NB) {
            int Js[NB], Ls[NB];
            rd4 t[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) {
              while (off >= nbk - L && L < nbk - 1) {
                off -= nbk - L;
                ++L;
              }
              Js[n] = L + off < nbk ? L + off : nbk - 1;
              Ls[n] = L;
              t[n] = tload(Js[n], Ls[n]);
              off += REJECT_T_TW;
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
              if (q + REJECT_T_TW * n < m) {
                tpad(t[n], Js[n], Ls[n]);
                tstore(tupd(t[n], Qp, Js[n], Ls[n]), Js[n], Ls[n]);
              }
            }
          }
        }
        // register tiles of block columns L > I
        const int Lr = I + 1 > L0 ? I + 1 : L0;
        if (Lr < nbk)
          for_slots(kfirst(t0r(Lr)), nslot, [&](int k, int J, int L) { tr[k] = tupd(tr[k], Qp, J, L); });
      }
      __syncthreads();   // (2)
      const int mask = sm.bmask;
      pmask = mask;
      if (mask == 0) continue;
      // 3. the panel below the block, as in the register-resident form
      const double* X = sm.XB[I & 1];
      for (int J = I + 1 + wt; J < nbk; J += REJECT_T_TW) {
        double av[4], bv[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          av[ks] = Qb[RT * J + l16][4 * ks + g];
          bv[ks] = X[l16 * RT + 4 * ks + g];
        }
        rd4 pj = rd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) pj = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv[ks], pj, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) Qb[RT * J + g + 4 * i][l16] = pj[i];
        if (RT * I + l16 < b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = RT * J + g + 4 * i;
            if (row < b) H[(int64_t)(RT * I + l16) * b + row] = pj[i];
          }
      }
      __syncthreads();   // (3)
      nacc += __popc(mask);
    }
  }
  __syncthreads();
  for (int a = tid; a < nacc; a += REJECT_T_THREADS) {
    const int64_t pv = props[sm.accl[a]];
    acc_out[a] = sm.accl[a];
    pivots[kr + a] = pv;
    u[pv] = 0.0;
  }
  if (tid == 0) st->s_r = nacc;
}

template <bool TAB>
__global__ __launch_bounds__(1024) void k_reject_global(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  double* __restrict__ H = RJ.H;
  const int b = RJ.b;
  const int64_t* __restrict__ props = RJ.props;
  const Unif un = ldc(RJ.un);
  RoundState* st = RJ.st;
  int32_t* __restrict__ acc_out = RJ.acc;
  int64_t* __restrict__ pivots = RJ.pivots;
  double* __restrict__ u = RJ.u;
  const int64_t kmax = RJ.kmax;
  const int keep_all = RJ.keep_all;
  if (st->status != ST_RUNNING) return;
  __shared__ unsigned char tk[BMAX];
  __shared__ short accl[BMAX];
  __shared__ int dec[2];
  __shared__ double sqv[2];
  FullGlobal S{H, b};
  reject_body(S, b, props, un, st, acc_out, pivots, u, kmax, keep_all, tk, dec, accl, sqv);
}

// --------------------------------------------------------- update preparation
// B operand of the update GEMM, Bt(c, j) = F(S_r(j), c) in the GEMM type
// (row-major, ld = ldb), and the accepted points Xp (s_r x d).
template <typename T>
__global__ __launch_bounds__(256) void k_prep(const double* __restrict__ Fs, int64_t ldf,
                                              const int32_t* __restrict__ acc, const int64_t* __restrict__ props,
                                              const double* __restrict__ X, int d,
                                              T* __restrict__ Bt, int ldb, double* __restrict__ Xp,
                                              const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int64_t kr = st->k_r;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < kr)
    for (int j = 0; j < s; ++j) Bt[c * ldb + j] = (T)Fs[(int64_t)acc[j] * ldf + c];
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < s * d; q += 256) {
      const int j = q / d, t = q % d;
      Xp[q] = X[props[acc[j]] * d + t];
    }
}

// Inverse of the s x s lower factor L (read from H through the accepted
// indices), one column per workgroup by forward substitution with wavefront
// dot products.  Writes
// Bt2(t, c) = Linv(c, t) in the GEMM type (row-major, ld b): the B operand of
// the triangular-solve product G = C Linv^T.
template <typename T>
__global__ __launch_bounds__(64) void k_trinv(LFactor L, T* __restrict__ Bt2, const RoundState* st) {
  const int b = L.b;
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int c = blockIdx.x;
  if (c >= s) return;
  __shared__ double x[BMAX];
  const int lane = threadIdx.x;
  for (int i = lane; i < s; i += 64) x[i] = 0.0;
  __syncthreads();
  if (lane == 0) x[c] = 1.0 / L.at(c, c);
  __syncthreads();
  for (int i = c + 1; i < s; ++i) {
    double p = 0.0;
    for (int t = c + lane; t < i; t += 64) p += L.at(i, t) * x[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
    if (lane == 0) x[i] = -p / L.at(i, i);
    __syncthreads();
  }
  // row c of Bt2 holds column c of Linv: Bt2(c, i) = Linv(i, c), zero for i < c
  for (int t = lane; t < s; t += 64) Bt2[(int64_t)c * b + t] = (t >= c) ? (T)x[t] : (T)0;
}

// ------------------------------------------------------------ diagonal update
// u <- max(u - rowsqnorm(G), 0) (Alg. 2 step 3) from the per-column-block
// partial row norms P (nparts x N, FP64, summed in a fixed order), and the
// new chunk sums.
template <bool TAB>
__global__ __launch_bounds__(CHUNK) void k_diag(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  double* __restrict__ u = RJ.u;
  double* __restrict__ csum = RJ.csum;
  const double* __restrict__ P = RJ.P;
  const int part_cols = RJ.part_cols;
  const int64_t N = RJ.N;
  const RoundState* st = RJ.st;
  if ((int64_t)blockIdx.x >= RJ.nchunks) return;
  if (st->status != ST_RUNNING || st->s_r == 0) return;
  __shared__ double sh[CHUNK];
  const int s = st->s_r;
  const int np = (s + part_cols - 1) / part_cols;
  const int64_t j = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double v = 0.0;
  if (j < N) {
    double g2 = 0.0;
    for (int q = 0; q < np; ++q) g2 += P[(int64_t)q * N + j];
    v = fmax(u[j] - g2, 0.0);
    u[j] = v;
  }
  const double t = block_sum<CHUNK>(v, sh);
  if (threadIdx.x == 0) csum[blockIdx.x] = t;
}

// End of round: k_r += s_r, round counters, stop conditions (k reached, an
// empty round, the round limit).
template <bool TAB>
__global__ void k_finish(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  RoundState* st = RJ.st;
  const int b = RJ.b;
  const int64_t kmax = RJ.kmax, max_rounds = RJ.max_rounds;
  int32_t* __restrict__ hist = RJ.hist;
  if (threadIdx.x != 0 || st->status != ST_RUNNING) return;
  const int s = st->s_r;
  hist[st->round] = s;
  st->k_r += s;
  st->round += 1;
  st->proposals += b;
  if (s == 0) st->status = ST_EARLY;
  else if (st->k_r >= kmax) st->status = ST_DONE;
  else if (max_rounds > 0 && st->round >= max_rounds) st->status = ST_DONE;
}

// Residual trace sum(u) from the chunk sums (end of run).
__global__ __launch_bounds__(1024) void k_trace(const double* __restrict__ csum, int64_t nchunks,
                                                double* __restrict__ out) {
  __shared__ double sh[1024];
  double v = 0.0;
  for (int64_t c = threadIdx.x; c < nchunks; c += 1024) v += csum[c];
  const double t = block_sum<1024>(v, sh);
  if (threadIdx.x == 0) *out = t;
}

// ------------------------------------------------------------------ launchers
void launch_trace(hipStream_t s, const double* csum, int64_t nchunks, double* out) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, s, csum, nchunks, out);
}

void launch_round_pack_e4m3(hipStream_t s, const double* X, int64_t N, int d, double* Xq, unsigned* X8, float* xn,
                            RoundState* st) {
  hipLaunchKernelGGL(k_round_pack_e4m3, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, X, N, d, Xq, X8, xn, st);
}

void launch_round_e4m3(hipStream_t s, const double* X, double* Xq, int64_t n) {
  const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_round_e4m3, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, X, Xq, n);
}

void launch_init(hipStream_t s, double* u, double* csum, const double* X, int64_t N, int d, KParams kp,
                 RoundState* st, int64_t nchunks) {
  hipLaunchKernelGGL(k_init, dim3((unsigned)nchunks), dim3(CHUNK), 0, s, u, csum, X, N, d, kp, st);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1024), 0, s, csum, nchunks, st);
}

void launch_init_from_diag(hipStream_t s, const double* u, int64_t N, double* csum, RoundState* st,
                           int64_t nchunks) {
  hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)nchunks), dim3(CHUNK), 0, s, u, N, csum);
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1024), 0, s, csum, nchunks, st);
}

void launch_propose(hipStream_t s, const double* u, const double* csum, double* cpre, int64_t nchunks,
                    int64_t N, int b, Unif un, RoundState* st, int64_t* props) {
  RoundJob j{};
  j.u = const_cast<double*>(u);
  j.csum = const_cast<double*>(csum);
  j.cpre = cpre;
  j.nchunks = nchunks;
  j.N = N;
  j.b = b;
  j.un = un;
  j.st = st;
  j.props = props;
  hipLaunchKernelGGL(k_scan_chunks<false>, dim3(1), dim3(1024), 0, s, j, nullptr);
  hipLaunchKernelGGL(k_propose<false>, dim3((b + PROPOSE_WAVES - 1) / PROPOSE_WAVES), dim3(64 * PROPOSE_WAVES), 0,
                     s, j, nullptr);
}

int gather_splits(int64_t kmax) {
  const int64_t p = (kmax + 255) / 256;
  return (int)(p < 1 ? 1 : (p > 8 ? 8 : p));
}

int64_t gather_width(int64_t kmax) {
  const int parts = gather_splits(kmax);
  return ((kmax + parts - 1) / parts + 63) / 64 * 64;
}

void launch_kernel_block(hipStream_t s, const double* X, int d, KParams kp, const int64_t* props, int b, double* H,
                         const RoundState* st) {
  RoundJob j{};
  j.X = X;
  j.d = d;
  j.kp = kp;
  j.props = const_cast<int64_t*>(props);
  j.b = b;
  j.parts = 0;
  j.Hp = nullptr;
  j.H = H;
  j.st = const_cast<RoundState*>(st);
  if (d > 32)
    hipLaunchKernelGGL(k_gather_Hs_tiled<false>, dim3((unsigned)(((b + HS_T - 1) / HS_T) * ((b + HS_T - 1) / HS_T))),
                       dim3(256), 0, s, j, nullptr);
  else
    hipLaunchKernelGGL(k_gather_Hs<false>, dim3((unsigned)(((int64_t)b * b + 255) / 256)), dim3(256), 0, s, j,
                       nullptr);
}

void launch_reject(hipStream_t s, double* H, int b, const int64_t* props, Unif un, RoundState* st,
                   int32_t* acc, int64_t* pivots, double* u, int64_t kmax, bool keep_all) {
  RoundJob j{};
  j.H = H;
  j.b = b;
  j.props = const_cast<int64_t*>(props);
  j.un = un;
  j.st = st;
  j.acc = acc;
  j.pivots = pivots;
  j.u = u;
  j.kmax = kmax;
  j.keep_all = keep_all ? 1 : 0;
  if (b <= REJECT_T_BMAX)
    hipLaunchKernelGGL((k_reject_tiled<false, false>), dim3(1), dim3(REJECT_T_THREADS), 0, s, j, nullptr);
  else if (b <= REJECT_G_BMAX)
    hipLaunchKernelGGL((k_reject_tiled<true, false>), dim3(1), dim3(REJECT_T_THREADS), 0, s, j, nullptr);
  else
    hipLaunchKernelGGL(k_reject_global<false>, dim3(1), dim3(1024), 0, s, j, nullptr);
}

// ---------------------------------------------- launchers over a table of jobs
RoundGrid round_grid_of(const RoundJob& j) {
  RoundGrid g{};
  g.propose = (unsigned)((j.b + PROPOSE_WAVES - 1) / PROPOSE_WAVES);
  g.gather_rows = (unsigned)(((j.kmax + 255) / 256) * j.b);
  const int64_t nb = (j.b + 15) / 16;
  g.gather_hp = (unsigned)(nb * nb * j.parts);
  g.gather_hs = j.d > 32 ? (unsigned)(((j.b + HS_T - 1) / HS_T) * ((j.b + HS_T - 1) / HS_T))
                         : (unsigned)(((int64_t)j.b * j.b + 255) / 256);
  g.diag = (unsigned)j.nchunks;
  return g;
}

void round_grid_max(RoundGrid& g, const RoundGrid& o) {
  g.propose = g.propose > o.propose ? g.propose : o.propose;
  g.gather_rows = g.gather_rows > o.gather_rows ? g.gather_rows : o.gather_rows;
  g.gather_hp = g.gather_hp > o.gather_hp ? g.gather_hp : o.gather_hp;
  g.gather_hs = g.gather_hs > o.gather_hs ? g.gather_hs : o.gather_hs;
  g.diag = g.diag > o.diag ? g.diag : o.diag;
}

void launch_propose_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g) {
  if (g.diag <= (unsigned)PS_MAXCH) {   // g.diag: the largest chunk count of the table
    hipLaunchKernelGGL(k_propose_scan<true>, dim3(g.propose, n), dim3(64 * PROPOSE_WAVES), 0, s, RoundJob{}, tab);
    return;
  }
  hipLaunchKernelGGL(k_scan_chunks<true>, dim3(1, n), dim3(1024), 0, s, RoundJob{}, tab);
  hipLaunchKernelGGL(k_propose<true>, dim3(g.propose, n), dim3(64 * PROPOSE_WAVES), 0, s, RoundJob{}, tab);
}

void launch_gather_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g, bool fdouble, bool tiled) {
  if (g.gather_rows > 0) {
    if (fdouble)
      hipLaunchKernelGGL((k_gather_rows<double, true>), dim3(g.gather_rows, n), dim3(256), 0, s, RoundJob{}, tab);
    else
      hipLaunchKernelGGL((k_gather_rows<float, true>), dim3(g.gather_rows, n), dim3(256), 0, s, RoundJob{}, tab);
  }
  if (fdouble)
    hipLaunchKernelGGL((k_gather_Hp<true, double>), dim3(g.gather_hp, n), dim3(64 * HP_WAVES), 0, s, RoundJob{}, tab);
  else
    hipLaunchKernelGGL((k_gather_Hp<true, float>), dim3(g.gather_hp, n), dim3(64 * HP_WAVES), 0, s, RoundJob{}, tab);
  if (tiled) hipLaunchKernelGGL(k_gather_Hs_tiled<true>, dim3(g.gather_hs, n), dim3(256), 0, s, RoundJob{}, tab);
  else hipLaunchKernelGGL(k_gather_Hs<true>, dim3(g.gather_hs, n), dim3(256), 0, s, RoundJob{}, tab);
}

void launch_reject_tab(hipStream_t s, const RoundJob* tab, int n, int bmax) {
  if (bmax <= REJECT_T_BMAX)
    hipLaunchKernelGGL((k_reject_tiled<false, true>), dim3(1, n), dim3(REJECT_T_THREADS), 0, s, RoundJob{}, tab);
  else if (bmax <= REJECT_G_BMAX)
    hipLaunchKernelGGL((k_reject_tiled<true, true>), dim3(1, n), dim3(REJECT_T_THREADS), 0, s, RoundJob{}, tab);
  else
    hipLaunchKernelGGL(k_reject_global<true>, dim3(1, n), dim3(1024), 0, s, RoundJob{}, tab);
}

void launch_diag_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g) {
  hipLaunchKernelGGL(k_diag<true>, dim3(g.diag, n), dim3(CHUNK), 0, s, RoundJob{}, tab);
}

void launch_finish_tab(hipStream_t s, const RoundJob* tab, int n) {
  hipLaunchKernelGGL(k_finish<true>, dim3(1, n), dim3(64), 0, s, RoundJob{}, tab);
}

template <typename T>
void launch_prep(hipStream_t s, const double* Fs, int64_t ldf, const int32_t* acc, const int64_t* props,
                 const double* X, int d, T* Bt, int ldb, double* Xp, const double* H, int b, T* Bt2,
                 int64_t kmax, const RoundState* st) {
  hipLaunchKernelGGL(k_prep<T>, dim3((unsigned)((kmax + 255) / 256)), dim3(256), 0, s, Fs, ldf, acc, props, X,
                     d, Bt, ldb, Xp, st);
  hipLaunchKernelGGL(k_trinv<T>, dim3(b), dim3(64), 0, s, LFactor{H, acc, b}, Bt2, st);
}
template void launch_prep<double>(hipStream_t, const double*, int64_t, const int32_t*, const int64_t*,
                                  const double*, int, double*, int, double*, const double*, int, double*,
                                  int64_t, const RoundState*);
template void launch_prep<float>(hipStream_t, const double*, int64_t, const int32_t*, const int64_t*,
                                 const double*, int, float*, int, double*, const double*, int, float*,
                                 int64_t, const RoundState*);

void launch_diag(hipStream_t s, double* u, double* csum, const double* P, int part_cols, int64_t N,
                 int64_t nchunks, const RoundState* st) {
  RoundJob j{};
  j.u = u;
  j.csum = csum;
  j.P = P;
  j.part_cols = part_cols;
  j.N = N;
  j.nchunks = nchunks;
  j.st = const_cast<RoundState*>(st);
  hipLaunchKernelGGL(k_diag<false>, dim3((unsigned)nchunks), dim3(CHUNK), 0, s, j, nullptr);
}

// Accepted points Xp(j, :) = X(S_r(j), :).
template <bool TAB>
__global__ __launch_bounds__(256) void k_prep_xp(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  prep_xp_range(RJ, st->s_r, (int)blockIdx.x, (int)gridDim.x);
}

// one element per thread (the gather is a chain of three dependent loads)
unsigned prep_xp_blocks(int64_t bd) {
  const int64_t g = (bd + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

void launch_prep_xp_tab(hipStream_t s, const RoundJob* tab, int n, int64_t bd) {
  hipLaunchKernelGGL(k_prep_xp<true>, dim3(prep_xp_blocks(bd), n), dim3(256), 0, s, RoundJob{}, tab);
}

// out[i] = the round state of table row i (out: host memory mapped for the
// device, so the host reads the states of a whole table after one event).
__global__ void k_collect_states(const RoundJob* __restrict__ tab, int n, RoundState* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *tab[i].st;
}

void launch_collect_tab(hipStream_t s, const RoundJob* tab, int n, RoundState* out) {
  hipLaunchKernelGGL(k_collect_states, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, tab, n, out);
}

// *dst = j: a job's table row written by a kernel (its argument is captured
// at launch, so the host copy need not outlive the call).
__global__ void k_store_job(RoundJob j, RoundJob* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = j;
}

void launch_store_job(hipStream_t s, const RoundJob& j, RoundJob* dst) {
  hipLaunchKernelGGL(k_store_job, dim3(1), dim3(64), 0, s, j, dst);
}

// End of a run enqueued without the host: columns k_r .. k-1 of F (element
// size es bytes, N rows) and pivots k_r .. k-1 (-1) as left by an early stop,
// read from the round state (nothing to do when k pivots are held).
__global__ __launch_bounds__(256) void k_zero_tail(const RoundState* __restrict__ st, int64_t k, int64_t N, int es,
                                                   void* __restrict__ F, int64_t* __restrict__ pivots) {
  const int64_t kr = st->k_r;
  if (kr >= k || st->nonfinite) return;
  const int64_t n = (k - kr) * N;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x, step = (int64_t)gridDim.x * 256;
  if (es == 8) {
    double* f = (double*)F + kr * N;
    for (int64_t i = i0; i < n; i += step) f[i] = 0.0;
  } else {
    float* f = (float*)F + kr * N;
    for (int64_t i = i0; i < n; i += step) f[i] = 0.f;
  }
  for (int64_t i = i0; i < k - kr; i += step) pivots[kr + i] = -1;
}

void launch_zero_tail(hipStream_t s, const RoundState* st, int64_t k, int64_t N, int es, void* F, int64_t* pivots) {
  hipLaunchKernelGGL(k_zero_tail, dim3(2048), dim3(256), 0, s, st, k, N, es, F, pivots);
}

void launch_finish(hipStream_t s, RoundState* st, int b, int64_t kmax, int64_t max_rounds, int32_t* hist) {
  RoundJob j{};
  j.st = st;
  j.b = b;
  j.kmax = kmax;
  j.max_rounds = max_rounds;
  j.hist = hist;
  hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(64), 0, s, j, nullptr);
}

}  // namespace arpc
