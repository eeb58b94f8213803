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
  const int64_t j = (int64_t)blockIdx.x * CHUNK + threadIdx.x;
  double v = 0.0;
  if (j < N) {
    v = kappa_r2(0.0, kp);
    u[j] = v;
    bool bad = false;
    for (int t = 0; t < d; ++t) bad |= !isfinite(X[j * d + t]);
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

template <bool TAB>
__global__ __launch_bounds__(64 * PROPOSE_WAVES) void k_propose(RoundJob j0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(j0, tab);
  const double* __restrict__ u = RJ.u;
  const double* __restrict__ cpre = RJ.cpre;
  const int64_t nchunks = RJ.nchunks, N = RJ.N;
  const int b = RJ.b;
  const Unif un = ldc(RJ.un);
  const RoundState* st = RJ.st;
  int64_t* __restrict__ props = RJ.props;
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
  const double base = (c > 0) ? cpre[c - 1] : 0.0;
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

// ------------------------------------------------------- gathers at proposals
typedef double rd4 __attribute__((ext_vector_type(4)));

// Fs(i, c) = F(props_i, c) in FP64, row-major with leading dimension ldf;
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
  Fs[(int64_t)i * ldf + c] = (double)F[c * N + props[i]];
}

// H = A(S',S') - F(S',:) F(S',:)^T (Alg. 2 step 2), FP64, column-major b x b
// (ld = b), in two launches.  First the product, split along the contraction
// index into partitions of W columns, on the FP64 matrix cores: workgroup
// (x, y, p) with x <= y forms the 16 x 16 tile of rows 16 y .., columns
// 16 x .. of partition p's partial product and writes it and its transpose
// into Hp(p) (workgroups above the diagonal have nothing to do).  Wavefront w
// contracts the 16-column chunks w, w + 4, .. of the partition as four
// 16x16x4 products (lane (g, l16) holds row l16 at column c + 4 g + m of
// product m); the four partial tiles are then added in wavefront order, so
// the result does not depend on scheduling, and a diagonal tile takes every
// entry from its lower half, so each Hp(p), and H, is exactly symmetric.
// The split keeps enough workgroups busy at any k_r.
template <bool TAB>
__global__ __launch_bounds__(256) void k_gather_Hp(RoundJob jb0, const RoundJob* __restrict__ tab) {
  ConstRoundJob& RJ = job_of<TAB>(jb0, tab);
  const int b = RJ.b;
  const double* __restrict__ Fs = RJ.Fs;
  const int64_t ldf = RJ.ldf, W = RJ.W;
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
  const double* ar = Fs + (int64_t)(ai ? i0 + l16 : 0) * ldf;
  const double* br = Fs + (int64_t)(bj ? j0 + l16 : 0) * ldf;
  rd4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c = cbeg + 16 * w; c < cend; c += 64) {
    double av[4], bv[4];
    if (c + 16 <= cend) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        av[m] = ai ? ar[c + 4 * g + m] : 0.0;
        bv[m] = bj ? br[c + 4 * g + m] : 0.0;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t k = c + 4 * g + m;
        av[m] = (ai && k < cend) ? ar[k] : 0.0;
        bv[m] = (bj && k < cend) ? br[k] : 0.0;
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv[m], acc, 0, 0, 0);
  }
  // entry e of lane (g, l16): row 16 y + g + 4 e, column 16 x + l16
  __shared__ double red[4][16][17];
#pragma unroll
  for (int e = 0; e < 4; ++e) red[w][g + 4 * e][l16] = acc[e];
  __syncthreads();
  const int r = tid >> 4, cc = tid & 15;
  const bool up = x == y && cc > r;
  const int rr = up ? cc : r, ck = up ? r : cc;
  const double v = ((red[0][rr][ck] + red[1][rr][ck]) + red[2][rr][ck]) + red[3][rr][ck];
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
  double sum = 0.0;
  for (int k0 = 0; k0 < d; k0 += HS_DC) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int r = sr + 4 * m;
      xs[r / HS_T][r % HS_T][sd] = k0 + sd < d ? src[m][k0 + sd] : 0.0;
    }
    __syncthreads();
    const int ke = d - k0 < HS_DC ? d - k0 : HS_DC;
    for (int t = 0; t < ke; ++t) {
      const double e = xs[0][ti][t] - xs[1][tj][t];
      sum += e * e;
    }
  }
  if (i < b && j < b) {
    const int64_t q = (int64_t)j * b + i;
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) acc += Hp[(int64_t)p * b * b + q];
    H[q] = kappa_r2(sum, kp) - acc;
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
// tiles in FP64 matrix-core accumulators (tile t = J (J + 1) / 2 + L of the
// lower triangle, J >= L, belongs to tile wavefront t mod 7; entry i of lane
// (g, n) is row 16 J + g + 4 i, column 16 L + n: the layout of the FP64
// 16x16x4 product's accumulator).  The proposals are taken 16 at a time
// (block column I), in this order in the GT form below:
//  1. the tile wavefronts finish the previous block's update on block column
//     I and copy it to LDS;
//  2. wavefront 0 runs the tests of Alg. 1 on the diagonal block while the
//     tile wavefronts apply the previous block's update to the rest of the
//     trailing tiles;
//  3. the panel below the block is solved against the accepted columns as a
//     product with the inverse of their factor, X (formed by wavefront 0 with
//     the tests), four matrix-core products per tile;
//  4. (at the next block) the trailing tiles receive the rank-16 update on
//     the matrix cores, four products per tile (rejected columns are zero).
// The register-resident form defers 3 and 4 of block I - 1 into block I
// (look-ahead): before block I's tests only the panel row P_I and the
// diagonal tile (I, I) are computed; the rest of the panel runs beside the
// first half of the tests and the rest of the update beside the second half
// (X double-buffered, barriers on LDS only).  The block-column buffer is
// double-buffered so a block's copy does not overwrite the previous panel
// while it is still being applied.  The scaled column of proposal i goes to
// column i of H (no longer read once in registers), where the solve's
// preparation reads it.
// For 256 < b <= 512 the triangle (up to 528 tiles, 1 MiB) does not fit the
// register file; the GT form keeps the trailing tiles in H and streams them
// through steps 1-4 (three full barriers per block; there the trailing
// update, not the tests, sets the pace, so the look-ahead gains nothing).
constexpr int RT = 16;                  // tile edge
constexpr int REJECT_T_THREADS = 512;
constexpr int REJECT_T_BMAX = 256;
constexpr int REJECT_G_BMAX = 512;      // the form with the trailing tiles in global memory
constexpr int REJECT_T_TW = 7;          // tile wavefronts
constexpr int REJECT_T_TPW = 20;        // tiles per tile wavefront: 136 / 7, rounded up
constexpr int QS = 18;                  // LDS row stride (doubles) of the block-column buffer

// (J, L) of lower-triangular tile index t, given those of t - step (L may
// start past J: it is carried into the following rows).
__device__ inline void tile_advance(int& J, int& L) {
  while (L > J) {
    L -= J + 1;
    ++J;
  }
}

// Workgroup barrier for LDS traffic only (it does not wait for global stores
// in flight): the register-resident form exchanges data between its waves
// only through LDS (the factor columns stored to H are read by later
// kernels, and every tile load from a column block of H has been consumed
// before that block's columns are written).
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
  __shared__ __attribute__((aligned(16))) double Q[2][BM][QS];  // block columns
  __shared__ double LD[RT][RT];            // LD[ii][r]: scaled accepted column ii at row r of the block
  __shared__ double BC[RT][RT];            // BC[ii][r]: column ii of the block when its test runs;
                                           // then X = L^{-1} of the block's accepted part, X(r, c) at BC[r][c]
  __shared__ double rsq[RT];               // 1/sqrt(h) of the accepted proposals (0: rejected)
  // register form (look-ahead): X of the last two blocks, XB[I & 1] for block I
  constexpr bool LA = !GT;
  __shared__ double XB[LA ? 2 * RT * RT : 1];
  __shared__ double uv[BM];     // u_i V_i of the test
  __shared__ int64_t pr[BM];
  __shared__ short prv[BM], accl[BM];
  __shared__ unsigned char tk[BM];
  __shared__ int bmask;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: tile coordinates stay scalar
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t kr = st->k_r, round = st->round;
  const int cap = (int)((kmax - kr) < b ? (kmax - kr) : b);
  const int nbk = (b + RT - 1) / RT;
  const int ntile = nbk * (nbk + 1) / 2;

  if (tid < b) {
    uv[tid] = keep_all ? 0.0 : H[(int64_t)tid * b + tid] * stream_uniform(un, 2 * (int64_t)b * round + b + tid);
    pr[tid] = props[tid];
    tk[tid] = 0;
  }
  __syncthreads();
  // the latest earlier proposal of the same point, eight LDS reads in flight
  if (tid < b) {
    const int64_t me = pr[tid];
    int p = -1;
    for (int q0 = tid - 1; q0 >= 0 && p < 0; q0 -= 8) {
      int64_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (q0 - k >= 0) ? pr[q0 - k] : -1;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (p < 0 && v[k] == me) p = q0 - k;
    }
    prv[tid] = (short)p;
  }

  int nacc = 0;
  if (w == 0) {
    // ---- the tests.  Lane r (mod 16) keeps row 16 I + r of the (symmetric)
    // diagonal block.  The update after an accepted proposal ii is written as
    // T(r, c) -= (T(r, ii) / h) T(c, ii), the same rank-one update as with the
    // scaled column, so the chain from one test to the next holds a
    // reciprocal but no square root; the scaled columns, 1/sqrt(h) and the
    // outputs are formed for the whole block afterwards, one lane per column.
    // Straight-line code: a rejected proposal has a zero multiplier.  Column
    // ii is broadcast through LDS at the start of its step, off the chain.
    // Lane ii also holds what the test of proposal 16 I + ii needs: u V, and
    // whether an earlier proposal of the same point was taken (before this
    // block: from tk; inside it: the scalar mask).
    int pm = 0;   // accepted columns of the previous block (register form: its panel is pending)
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      double(*Qb)[QS] = Q[I & 1];
      if constexpr (LA) {
        lds_sync();   // (1) the diagonal block of block column I is in LDS
      } else {
        __syncthreads();   // (1) block column I is in LDS
      }
      double dr[RT];
#pragma unroll
      for (int c = 0; c < RT; ++c) dr[c] = Qb[RT * I + l16][c];
      const int iL = RT * I + l16;
      double uvL = 0.0;
      int pL = -1;
      bool dupL = false;
      if (iL < b) {
        uvL = uv[iL];
        const int p = prv[iL];
        if (p >= RT * I) pL = p - RT * I;
        else if (p >= 0) dupL = tk[p] != 0;
      }
      const unsigned dup_before = (unsigned)__ballot(dupL) & 0xffffu;
      int mask = 0, taken = 0, cnt = 0;
      double hL = 1.0;   // lane ii: h of proposal 16 I + ii
#pragma unroll
      for (int ii = 0; ii < RT; ++ii) {
        const int i = RT * I + ii;
        if constexpr (LA) {
          if (ii == RT / 2 && pm) lds_sync();   // (m)
        }
        // column ii is final: T(ii + 1, ii), needed by the next test, by
        // readlane; the rest through LDS (lanes r and r + 16 k write the same
        // value), needed no earlier than the test after next
        BC[ii][l16] = dr[ii];
        const double bn = readlane_f64(dr[ii], ii + 1 < RT ? ii + 1 : ii);
        double bc[RT];
#pragma unroll
        for (int c = ii + 2; c < RT; ++c) bc[c] = BC[ii][c];
        // the test, evaluated on lane ii (which holds h = its diagonal entry)
        const int dupl = (int)((dup_before >> l16) & 1u) | ((pL >= 0) & (int)((taken >> (pL & 15)) & 1));
        const int al = (dupl ^ 1) & (uvL < dr[ii] ? 1 : 0);
        const int bits = __builtin_amdgcn_readlane(al | (dupl << 1), ii);
        const bool dup = (bits & 2) != 0;
        const bool a = (bits & 1) && i < b && nacc + cnt < cap;
        const double h = readlane_f64(dr[ii], ii);
        taken |= (a || dup) ? (1 << ii) : 0;
        // 1/h: hardware reciprocal and two Newton steps (exact for h = 1)
        const double ha = a ? h : 1.0;
        double inv = __builtin_amdgcn_rcp(ha);
        inv = fma(inv, fma(-ha, inv, 1.0), inv);
        inv = fma(inv, fma(-ha, inv, 1.0), inv);
        const double t = a ? dr[ii] * inv : 0.0;
        if (ii + 1 < RT) dr[ii + 1] = fma(-t, bn, dr[ii + 1]);
#pragma unroll
        for (int c = ii + 2; c < RT; ++c) dr[c] = fma(-t, bc[c], dr[c]);
        hL = (l16 == ii) ? h : hL;
        mask |= a ? (1 << ii) : 0;
        cnt += a ? 1 : 0;
      }
      // the block's outputs: lane c forms 1/sqrt(h_c); row r keeps the
      // unscaled entries T(r, ii) of the steps, which scale into column ii
      const double rsL = ((mask >> l16) & 1) ? 1.0 / sqrt(hL) : 0.0;
      if (lane < RT) {
        rsq[lane] = rsL;
        if (iL < b) tk[iL] = (taken >> lane) & 1;
        if ((mask >> lane) & 1) accl[nacc + __popc(mask & ((1 << lane) - 1))] = (short)iL;
      }
      double rs[RT];
#pragma unroll
      for (int ii = 0; ii < RT; ++ii) rs[ii] = rsq[ii];
      // column ii of the factor (zero for a rejected proposal) into column
      // 16 I + ii of H, rows of the block at and below ii
#pragma unroll
      for (int ii = 0; ii < RT; ++ii) {
        const double col = (l16 >= ii) ? dr[ii] * rs[ii] : 0.0;
        if (lane < RT) LD[ii][lane] = col;
        if (lane < RT && lane >= ii && iL < b && RT * I + ii < b) H[(int64_t)(RT * I + ii) * b + iL] = col;
      }
      // X = L^{-1} restricted to the accepted proposals (rejected rows and
      // columns come out zero): lane c forms column c by forward
      // substitution, into XS(r, c) (the broadcast area, free again)
      {
        double y[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) y[r] = (r == l16) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < RT; ++k) {
          const double xk = y[k] * rsq[k];
          y[k] = xk;
#pragma unroll
          for (int r = k + 1; r < RT; ++r) y[r] = fma(-LD[k][r], xk, y[r]);
        }
        double* xo = LA ? XB + (I & 1) * RT * RT : &BC[0][0];
        if (lane < RT)
#pragma unroll
          for (int r = 0; r < RT; ++r) xo[r * RT + lane] = y[r];
      }
      if (lane == 0) bmask = mask;
      if constexpr (LA) {
        lds_sync();   // (2) decisions, LD, rsq and X are in LDS
        pm = mask;
        if (mask == 0) continue;
      } else {
        __syncthreads();   // (2) decisions, LD, rsq and X are in LDS
        if (mask == 0) continue;
        __syncthreads();   // (3) the panel is solved
      }
      nacc += __popc(mask);
    }
  } else if constexpr (!GT) {
    const int wt = w - 1;
    rd4 tr[REJECT_T_TPW];
    // coordinates of this wavefront's tiles, four bits each of J and L, four
    // tiles per word (scalar registers)
    unsigned pk[(REJECT_T_TPW + 3) / 4];
    {
#pragma unroll
      for (int q = 0; q < (REJECT_T_TPW + 3) / 4; ++q) pk[q] = 0;
      int J = 0, L = wt;
#pragma unroll
      for (int k = 0; k < REJECT_T_TPW; ++k) {
        tile_advance(J, L);
        pk[k / 4] |= (unsigned)((J & 15) | ((L & 15) << 4)) << (8 * (k % 4));
        L += REJECT_T_TW;
      }
    }
    // f(k, J, L) for each tile k of this wavefront
    auto for_tiles = [&](auto f) __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < REJECT_T_TPW; ++k) {
        if (wt + REJECT_T_TW * k < ntile) {
          const unsigned e = pk[k / 4] >> (8 * (k % 4));
          f(k, (int)(e & 15), (int)((e >> 4) & 15));
        }
      }
    };
    // this wavefront's tiles of H (zero padding), read along rows of the
    // symmetric H so that a load instruction covers four 128-byte runs; the
    // loads are unconditional (clamped indices) so that all stay in flight
#pragma unroll
    for (int k = 0; k < REJECT_T_TPW; ++k) tr[k] = rd4{0.0, 0.0, 0.0, 0.0};
    for_tiles([&](int k, int J, int L) {
      const int col = RT * L + l16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = RT * J + g + 4 * i;
        tr[k][i] = H[(int64_t)(row < b ? row : b - 1) * b + (col < b ? col : b - 1)];
      }
    });
    for_tiles([&](int k, int J, int L) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (RT * J + g + 4 * i >= b || RT * L + l16 >= b) tr[k][i] = 0.0;
    });
    // T(J, L) -= P_J P_L^T for the tiles selected by pick(J, L), four k-steps
    // of four columns (rejected columns of P are zero), P the previous block's
    // solved panel; a tile's eight operands are read before its products
    auto update2 = [&](double(*P)[QS], auto pick) __attribute__((always_inline)) {
      for_tiles([&](int k, int J, int L) {
        if (__builtin_expect(pick(J, L), 0)) {
          double av[4], bv[4];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            av[ks] = P[RT * J + l16][4 * ks + g];
            bv[ks] = P[RT * L + l16][4 * ks + g];
          }
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) tr[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[ks], bv[ks], tr[k], 0, 0, 0);
        }
      });
    };
    // tiles selected by pick(J, L) into the rows of block J of the buffer
    auto copy_to = [&](double(*Qd)[QS], auto pick) __attribute__((always_inline)) {
      for_tiles([&](int k, int J, int L) {
        if (__builtin_expect(pick(J, L), 0))
#pragma unroll
          for (int i = 0; i < 4; ++i) Qd[RT * J + g + 4 * i][l16] = tr[k][i];
      });
    };
    // panel rows J >= Jlo of block Ip (spread: row J to tile wavefront
    // (J - Jlo) mod 7; else row Jlo only, by the caller): P_J = Q_J X^T from the copy of block column Ip, in place, and the
    // accepted columns into H.  A loop over J, not over this wavefront's tiles
    // (it touches no tile registers).
    auto panel = [&](double(*Qs)[QS], const double* X, int Ip, int Jlo, bool spread) __attribute__((always_inline)) {
      const int j0 = spread ? Jlo + wt : Jlo, je = spread ? nbk : Jlo + 1;
      for (int J = j0; J < je; J += REJECT_T_TW) {
        rd4 pj = rd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          pj = __builtin_amdgcn_mfma_f64_16x16x4f64(Qs[RT * J + l16][4 * ks + g], X[l16 * RT + 4 * ks + g], pj, 0,
                                                    0, 0);
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
    // diagonal tile (I, I) are computed (by that tile's owner); the rest of
    // the panel runs beside the first half of the tests and the rest of the
    // update beside the second half, the block's outputs and its inverse
    // factor (wavefront 0 takes the barrier (m) between them inside its test
    // loop).
    int pmask = 0;   // accepted columns of the previous block (panel and update pending)
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      double(*Qb)[QS] = Q[I & 1];
      double(*Qp)[QS] = Q[(I + 1) & 1];         // block column I - 1, becoming its panel
      const double* Xp = XB + ((I + 1) & 1) * RT * RT;   // X of block I - 1
      if (pmask) {
        // panel row I of block I - 1 (P_I = Q_I X^T), by the owner of the
        // diagonal tile (I, I), which then updates that tile with it (its own
        // LDS writes are ordered before its reads); the other waves read P_I
        // only after (m)
        if ((I * (I + 1) / 2 + I) % REJECT_T_TW == wt) {
          panel(Qp, Xp, I - 1, I, false);
          update2(Qp, [&](int J, int L) { return J == I && L == I; });
        }
      }
      copy_to(Qb, [&](int J, int L) { return J == I && L == I; });
      lds_sync();   // (1)
      if (pmask) {
        panel(Qp, Xp, I - 1, I + 1, true);
        lds_sync();   // (m)
        update2(Qp, [&](int J, int L) { return L >= I && !(J == I && L == I); });
      }
      copy_to(Qb, [&](int J, int L) { return L == I && J > I; });
      lds_sync();   // (2)
      const int mask = bmask;
      pmask = mask;
      if (mask == 0) continue;
      nacc += __popc(mask);
    }
  } else {
    // Trailing tiles in H itself: tile (J, L), J >= L, element (r, c) (row
    // 16 J + r, column 16 L + c of the residual) at H[(16 J + r) b + 16 L + c],
    // which is the upper triangle of the column-major H for J > L and the
    // whole diagonal block for J = L.  The factor goes to the lower triangle
    // of block columns already consumed, so the two never overlap.  At most
    // 2 MiB, held in the L2 of the workgroup's XCD; each update is a load,
    // four matrix-core products and a store per tile.
    const int wt = w - 1;
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
    constexpr int NB = 8;                                                       // tiles in flight in the update
    int pmask = 0;
    for (int I = 0; I < nbk && nacc < cap; ++I) {
      double(*Qb)[QS] = Q[I & 1];
      double(*Qp)[QS] = Q[(I + 1) & 1];
      // 1. block column I (tiles (J, I), J >= I) with the pending update, to LDS
      {
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
      }
      __syncthreads();   // (1)
      // 2. the rest of the pending update, beside the tests: the trailing
      // tiles (J, L), J >= L > I, numbered down the block columns, tile q to
      // tile wavefront q mod 7, eight loads in flight
      if (pmask) {
        const int nt = nbk - I - 1, m = nt * (nt + 1) / 2;
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
      __syncthreads();   // (2)
      const int mask = bmask;
      pmask = mask;
      if (mask == 0) continue;
      // 3. the panel below the block, as in the register-resident form
      for (int J = I + 1 + wt; J < nbk; J += REJECT_T_TW) {
        double av[4], bv[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          av[ks] = Qb[RT * J + l16][4 * ks + g];
          bv[ks] = BC[l16][4 * ks + g];
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
    const int64_t pv = props[accl[a]];
    acc_out[a] = accl[a];
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
  hipLaunchKernelGGL(k_gather_Hp<true>, dim3(g.gather_hp, n), dim3(256), 0, s, RoundJob{}, tab);
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
  const int32_t* __restrict__ acc = RJ.acc;
  const int64_t* __restrict__ props = RJ.props;
  const double* __restrict__ X = RJ.X;
  const int d = RJ.d;
  double* __restrict__ Xp = RJ.Xp;
  const RoundState* st = RJ.st;
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < s * d; q += gridDim.x * 256) {
    const int j = q / d, t = q % d;
    Xp[q] = X[props[acc[j]] * d + t];
  }
}

void launch_prep_xp(hipStream_t s, const int32_t* acc, const int64_t* props, const double* X, int d, double* Xp,
                    const RoundState* st) {
  RoundJob j{};
  j.acc = const_cast<int32_t*>(acc);
  j.props = const_cast<int64_t*>(props);
  j.X = X;
  j.d = d;
  j.Xp = Xp;
  j.st = const_cast<RoundState*>(st);
  hipLaunchKernelGGL(k_prep_xp<false>, dim3(8), dim3(256), 0, s, j, nullptr);
}

void launch_prep_xp_tab(hipStream_t s, const RoundJob* tab, int n) {
  hipLaunchKernelGGL(k_prep_xp<true>, dim3(8, n), dim3(256), 0, s, RoundJob{}, tab);
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
