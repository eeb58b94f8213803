// Internal definitions shared by the kernels and the host code of the
// accelerated RPCholesky library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arpc {

// Rows per residual-diagonal chunk.  The diagonal-update kernel writes one
// partial sum per chunk; the proposal kernel scans the chunk sums and then the
// elements of a single chunk per draw.
constexpr int CHUNK = 1024;
// Largest block size.  The b x b residual submatrix is FP64 in global memory
// (8 MiB at b = 1024); RejectionSampleSubmatrix keeps its trailing tiles in
// registers for b <= 256, in L2 for b <= 512, and runs on the full matrix in
// global memory above that (one workgroup of 1024 threads).
constexpr int BMAX = 1024;

enum : int32_t { ST_RUNNING = 0, ST_DONE = 1, ST_EARLY = 2, ST_NOUNIF = 3 };

// Device-resident round state; every round kernel reads it so that the host
// never has to synchronise inside a round.
struct RoundState {
  int64_t k_r;        // pivots held at the start of the current round
  int64_t round;      // rounds completed
  int64_t proposals;  // proposals consumed
  int32_t s_r;        // pivots accepted in the current round
  int32_t status;     // ST_*
  double T;           // residual trace at the start of the current round
  double trace_A;     // sum of diag A
  int32_t nonfinite;  // set if a point has a NaN/Inf coordinate
  int32_t lastpos;    // last chunk with a positive sum (proposal rounding fallback)
};

// Source of the uniform stream: explicit array (U != nullptr) or Philox keyed by seed.
struct Unif {
  const double* U;
  int64_t nU;
  uint64_t seed;
};

struct KParams {
  int kernel;
  double sigma;
  double c0;  // kernel-specific constant (see kappa_r2)
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

// Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11), counter
// (q+1, 0, 0, 0) for block q, key (seed, 0); returns word p = 4q + (p mod 4).
__host__ __device__ inline uint64_t philox_word(uint64_t seed, uint64_t p) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = (p >> 2) + 1, x1 = 0, x2 = 0, x3 = 0;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = mulhi64(M0, x0), lo0 = M0 * x0;
    const uint64_t hi1 = mulhi64(M1, x2), lo1 = M1 * x2;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  const uint64_t w[4] = {x0, x1, x2, x3};
  return w[p & 3];
}

__host__ __device__ inline double philox_uniform(uint64_t seed, uint64_t p) {
  return (double)(philox_word(seed, p) >> 11) * 0x1.0p-53;
}

__device__ inline double stream_uniform(const Unif& un, int64_t p) {
  if (un.U) return un.U[p];
  return philox_uniform(un.seed, (uint64_t)p);
}

// Kernel value from the squared distance, in FP64 (Section 1.2 Gaussian;
// Laplace with the l2 distance; Matern-3/2; Matern-5/2 of Section 3.2).
__device__ __attribute__((always_inline)) inline double kappa_r2(double r2, const KParams& kp) {
  switch (kp.kernel) {
    case 0: return exp(-r2 * kp.c0);                 // c0 = 1/(2 sigma^2)
    case 1: return exp(-sqrt(r2) / kp.sigma);
    case 2: {
      const double t = 1.7320508075688772 * sqrt(r2) / kp.sigma;
      return (1.0 + t) * exp(-t);
    }
    default: {
      const double t = 2.23606797749979 * sqrt(r2) / kp.sigma;
      return (1.0 + t + r2 * kp.c0) * exp(-t);       // c0 = 5/(3 sigma^2)
    }
  }
}

// The same kernel values in FP32 (used by the reduced-precision modes).
__device__ __attribute__((always_inline)) inline float kappa_r2_f32(float r2, const KParams& kp) {
  switch (kp.kernel) {
    case 0: return expf(-r2 * (float)kp.c0);
    case 1: return expf(-sqrtf(r2) / (float)kp.sigma);
    case 2: {
      const float t = 1.7320508f * sqrtf(r2) / (float)kp.sigma;
      return (1.0f + t) * expf(-t);
    }
    default: {
      const float t = 2.2360680f * sqrtf(r2) / (float)kp.sigma;
      return (1.0f + t + r2 * (float)kp.c0) * expf(-t);
    }
  }
}

// The four kernels in one branch-free FP32 form (for the fused BF16-mode
// epilogue, where a per-element switch would multiply the code by four):
//   t = scale * (use_r ? |x - y| : |x - y|^2),
//   kappa = (1 + p1 t + p2 t^2) * 2^(-q t).
// Gaussian: t = r^2 / (2 s^2), p1 = p2 = 0; Laplace: t = r / s, p1 = p2 = 0;
// Matern-3/2: t = sqrt3 r / s, p1 = 1, p2 = 0; Matern-5/2: t = sqrt5 r / s,
// p1 = 1, p2 = 1/3 (Section 1.2, Section 3.2).  q = log2(e).
struct KFast {
  float scale, p1, p2, q;
  int use_r;
};

__host__ inline KFast kfast_of(const KParams& kp) {
  KFast k{};
  k.q = 1.4426950408889634f;
  const double s = kp.sigma;
  switch (kp.kernel) {
    case 0: k.scale = (float)(1.0 / (2.0 * s * s)); k.use_r = 0; break;
    case 1: k.scale = (float)(1.0 / s); k.use_r = 1; break;
    case 2: k.scale = (float)(1.7320508075688772 / s); k.use_r = 1; k.p1 = 1.f; break;
    default: k.scale = (float)(2.23606797749979 / s); k.use_r = 1; k.p1 = 1.f; k.p2 = 1.f / 3.f; break;
  }
  return k;
}

__device__ __attribute__((always_inline)) inline float kappa_fast(float r2, const KFast& k) {
  const float u = k.use_r ? __builtin_amdgcn_sqrtf(r2) : r2;
  const float t = u * k.scale;
  const float poly = fmaf(fmaf(k.p2, t, k.p1), t, 1.0f);
  return poly * __builtin_amdgcn_exp2f(-k.q * t);
}

// Arguments of the one-kernel round product of the BF16 modes (see
// fused_kernels.hip).
struct FusedArgs {
  const __bf16* Fb;         // panel-blocked BF16 planes of F
  int64_t nkc;              // chunks per panel of Fb
  int64_t N;
  const unsigned char* Bm1; // F(S_r,:)^T in chunks
  const unsigned char* Bm2; // permuted inverse factor in chunks
  const double* X;          // N x d
  int d;
  const double* Xp;         // s_r x d accepted points
  KFast kf;
  float* Fu;                // F, column-major, ld N
  __bf16* Fbw;              // Fb (written)
  double* P;                // row norms of G
  const RoundState* st;
  int ntiles;
};

// Device pointers and sizes of one factorization that the round kernels read
// (the proposals, the residual submatrix, RejectionSampleSubmatrix, the
// accepted points, the diagonal update, the round control and, in the BF16
// modes, the one-kernel round product).  Every such kernel takes a table of
// these and serves the factorization in row blockIdx.y of the table, so one
// launch can advance the rounds of several factorizations (serving), or of
// one (a table of one row).  Per-round values (k_r, s_r, the round) are read
// from the round state, so a table row does not change during a run.
struct RoundJob {
  RoundState* st;
  double* u;              // residual diagonal (N)
  double* csum;           // its chunk sums
  double* cpre;           // their inclusive prefix
  int64_t nchunks;
  int64_t N;
  const double* X;        // N x d points, row-major (the rounded copy in the FP8 mode)
  int d;
  int b;
  Unif un;
  KParams kp;
  int64_t* props;         // b proposals
  int32_t* acc;           // accepted local indices
  int64_t* pivots;        // k outputs
  int64_t kmax;           // k
  int64_t max_rounds;
  int keep_all;           // block RPCholesky (Alg. 7)
  int part_cols;          // columns per partial row-norm group of P
  const void* F;          // N x k column-major factor (FP64 or FP32)
  double* Fs;             // F rows at the proposals, FP64, ld ldf
  float* Fs32;            // the same rows in FP32 (F stored in FP32), else null; ld fs32_ld(ldf)
  int64_t ldf;
  double* Hp;             // partial products of F(S',:) F(S',:)^T
  int64_t W;              // contraction columns per partition of Hp
  int parts;
  double* H;              // b x b residual submatrix, then L(T,T)
  double* Xp;             // accepted points
  const double* P;        // partial row norms of G
  int32_t* hist;          // accepted count per round
  const void* Fb;         // BF16 modes: panel-blocked copy of F
  int64_t nkc;
  unsigned char* Bm1;
  unsigned char* Bm2;
  int CP;                 // padded column count of the round product
  int nt;                 // 32-column chunks of the inverse factor
  FusedArgs fa;
};

// Leading dimension of the FP32 copy of F(S',:): a multiple of four, so four
// consecutive entries of a row are one aligned 16-byte load.
__host__ __device__ inline int64_t fs32_ld(int64_t ldf) { return (ldf + 3) & ~(int64_t)3; }

// A table row read as kernel arguments are: through the constant address
// space, so the compiler uses scalar loads into scalar registers (the table
// is written before the launch and not changed by it).
typedef const __attribute__((address_space(4))) RoundJob ConstRoundJob;

__device__ __forceinline__ ConstRoundJob& table_row(const RoundJob* tab) {
  return ((ConstRoundJob*)tab)[blockIdx.y];
}

// A copy of a member of such a row (a struct), word by word through the
// constant address space.
template <class T>
__device__ __forceinline__ T ldc_any(const T& x) { return x; }

template <class T>
__device__ __forceinline__ T ldc(const __attribute__((address_space(4))) T& x) {
  static_assert(sizeof(T) % 4 == 0, "word copy");
  T v;
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)&x;
  uint32_t* dst = (uint32_t*)&v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
  return v;
}

template <class T>
__device__ __forceinline__ T ldc_any(const __attribute__((address_space(4))) T& x) { return ldc(x); }

// The table row of this workgroup (TAB), or the single job passed by value.
template <bool TAB>
__device__ __forceinline__ ConstRoundJob& job_of(const RoundJob& j0, const RoundJob* tab) {
  if constexpr (TAB) return table_row(tab);
  else return *(ConstRoundJob*)&j0;
}

__device__ inline double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// The accepted factor L(T,T) as RejectionSampleSubmatrix leaves it: entry
// (a, c), a >= c, is H(acc[a], acc[c]) (the scaled column of proposal acc[c]
// stays in column acc[c] of the b x b column-major H).  Entries above the
// diagonal are not defined.
struct LFactor {
  const double* H;
  const int32_t* acc;
  int b;
  __device__ double at(int a, int c) const { return H[(int64_t)acc[c] * b + acc[a]]; }
};

// Column c of the inverse of the s x s lower-triangular L, s <= 64 M, in one
// wavefront by column-oriented forward substitution: lane l keeps rows l,
// l + 64, ..., l + 64 (M - 1) of the right-hand side e_c, which becomes
// column c of L^{-1}.  Column t of L (gathered from one column of H) does not
// depend on the solution, so it is loaded P steps ahead (an L2 round trip per
// step otherwise); the dependency chain is one readlane and a few FMAs per
// step.  Rows outside [c, s) are zero.
template <int M>
__device__ inline void linv_column(const LFactor& L, int s, int c, int lane, double (&r)[M]) {
  constexpr int P = 8;   // columns of L in flight ahead of the chain (divides 64)
  double invd[M];
  int64_t ic[M];         // H row of row i (clamped to s - 1; rows outside (t, s) are masked at use)
  if (c >= s) {
#pragma unroll
    for (int m = 0; m < M; ++m) r[m] = 0.0;
    return;
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int i = lane + 64 * m;
    r[m] = (i == c) ? 1.0 : 0.0;
    invd[m] = (i < s) ? 1.0 / L.at(i, i) : 0.0;
    ic[m] = L.acc[i < s ? i : s - 1];
  }
  // Steps t run from c rounded down to a multiple of P (earlier ones are
  // skipped); column t of L sits in buf[t % P], loaded P steps ahead with an
  // unconditional load (column index clamped to s - 1).  The rows of step t
  // live in register group t / 64 of lane t % 64; the M groups are walked
  // in turn, so that group is a compile-time choice and only groups at or
  // past it are updated.
  const int t0 = c & ~(P - 1);
  double buf[P][M];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    const int tc = t0 + u < s ? t0 + u : s - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) buf[u][m] = L.H[(int64_t)L.acc[tc] * L.b + ic[m]];
  }
  int t = t0;
#pragma unroll
  for (int mt = 0; mt < M; ++mt) {
    const int te = s < 64 * (mt + 1) ? s : 64 * (mt + 1);
    for (; t < te; t += P) {
#pragma unroll
      for (int u = 0; u < P; ++u) {
        const int tt = t + u;
        if (tt >= c && tt < te) {
          const int lt = tt & 63;
          const double xt = readlane_f64(r[mt], lt) * readlane_f64(invd[mt], lt);
          r[mt] = (lane == lt) ? xt : r[mt];
#pragma unroll
          for (int m = mt; m < M; ++m) {
            const int i = lane + 64 * m;
            const double lv = (i > tt && i < s) ? buf[u][m] : 0.0;   // rows tt+1 .. s-1 of column tt
            r[m] = fma(-lv, xt, r[m]);
          }
        }
        const int tn = tt + P < s ? tt + P : s - 1;
#pragma unroll
        for (int m = 0; m < M; ++m) buf[u][m] = L.H[(int64_t)L.acc[tn] * L.b + ic[m]];
      }
    }
  }
}

// Largest b whose RejectionSampleSubmatrix runs in the tiled form, which also
// leaves the inverses of its 16 x 16 diagonal blocks in H (see linv_blocks_ahead).
constexpr int REJECT_TILED_BMAX = 512;

// Column c of the inverse of the accepted factor L(T,T) (s x s), in proposal
// indexing: x[q] = (L(T,T)^{-1})(i, c) at q = acc[i], zero at every proposal
// that was not accepted.  Block forward substitution over the 16-proposal
// blocks of the tiled RejectionSampleSubmatrix, which leaves in H the factor
// columns (lower triangle, proposal indexing, columns of rejected proposals
// zero) and, in the upper triangle of each diagonal block J, the strictly
// lower part of the inverse X_J of that block's accepted factor (X_J(r, q) at
// H[(16 J + r) b + 16 J + q], r > q; its diagonal is 1 / H(p, p), zero where
// that column is zero).  With p = acc[c] and e = e_p,
//   x_J = X_J (e_J - sum_{K < J} L_JK x_K),  J = block(p) .. block(acc[s - 1]),
// so the chain is one step per block, not per proposal.
// On NW wavefronts, each block's operands loaded one block ahead: the loads
// of step J + 1 (its row of L blocks and X_{J+1}) go out before the
// arithmetic of step J, so the chain waits for about one L2 round trip in all
// instead of one per block.  Lane (w, g, r) of the 64 NW takes row r of a
// block and the blocks K = J0 + 4 w + g + 4 NW t (t < 2: at most 8 NW + 1
// blocks); the wavefronts' partial sums meet in ysum (2 x NW x 16 doubles of
// LDS, by step parity), one barrier per step, and every wavefront then forms
// x_J (the same values in the same order) and stores it.  x: b doubles of
// LDS.  Every thread of the workgroup must call it.
template <int NW>
__device__ __attribute__((always_inline)) inline void linv_blocks_ahead(const double* __restrict__ H,
                                                                        const int32_t* __restrict__ acc, int b, int s,
                                                                        int c, int tid, double* x, double* ysum) {
  constexpr int KS = 2;
  const int lane = tid & 63, w = tid >> 6, g = lane >> 4, r = lane & 15;
  const int p = acc[c];
  const int J0 = p >> 4, J1 = acc[s - 1] >> 4;
  for (int i = tid; i < b; i += 64 * NW) x[i] = 0.0;
  __syncthreads();
  struct Ops {
    double l[KS][16];   // L_JK(r, q) for K = J0 + 4 w + g + 4 NW t < J
    double xq[4];       // X_J(r, 4 g + j) below the diagonal, H(row, row) on it
  };
  auto load = [&](Ops& o, int J) __attribute__((always_inline)) {
    const int row = 16 * J + r;
    const int rowc = row < b ? row : b - 1;
    // a uniform base per column q and one 32-bit offset per lane and block
    // (b <= 8 NW + 1 blocks: every offset fits), so the addresses cost no
    // registers per load
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int K = J0 + 4 * w + g + 4 * NW * t;
      const unsigned off = (unsigned)(16 * K * b + rowc);
      if (K < J) {
#pragma unroll
        for (int q = 0; q < 16; ++q) o.l[t][q] = (H + q * b)[off];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * g + j;
      double v = 0.0;
      if (row < b && 16 * J + q < b && q <= r) v = H[(unsigned)(row * b + (q < r ? 16 * J + q : row))];
      o.xq[j] = v;
    }
  };
  auto step = [&](const Ops& o, int J) __attribute__((always_inline)) {
    const int row = 16 * J + r;
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const int K = J0 + 4 * w + g + 4 * NW * t;
      if (K < J) {
#pragma unroll
        for (int q = 0; q < 16; q += 2) {
          t0 = fma(o.l[t][q], x[16 * K + q], t0);
          t1 = fma(o.l[t][q + 1], x[16 * K + q + 1], t1);
        }
      }
    }
    double y = t0 + t1;
    y += __shfl_xor(y, 16, 64);
    y += __shfl_xor(y, 32, 64);
    double* ys = ysum + (J & 1) * (16 * NW);
    if (g == 0) ys[w * 16 + r] = y;
    __syncthreads();
    double ya = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) ya += ys[16 * v + r];
    y = (row == p ? 1.0 : 0.0) - ya;
    double xr = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * g + j;
      const double yq = __shfl(y, q, 64);
      const double xq = q < r ? o.xq[j] : (q == r && o.xq[j] > 0.0 ? 1.0 / o.xq[j] : 0.0);
      xr = fma(xq, yq, xr);
    }
    xr += __shfl_xor(xr, 16, 64);
    xr += __shfl_xor(xr, 32, 64);
    if (g == 0 && row < b) x[row] = xr;
  };
  Ops a, bb;
  load(a, J0);
  for (int J = J0; J <= J1; J += 2) {
    if (J + 1 <= J1) load(bb, J + 1);
    step(a, J);
    if (J + 1 > J1) break;
    if (J + 2 <= J1) load(a, J + 2);
    step(bb, J + 1);
  }
}

// Accepted points Xp(j, :) = X(S_r(j), :), element q = j d + t taken by
// virtual workgroup vb of vg (256 threads each): one element per thread,
// since each is a chain of three dependent loads.
__device__ __attribute__((always_inline)) inline void prep_xp_range(ConstRoundJob& RJ, int s, int vb, int vg) {
  const int32_t* __restrict__ acc = RJ.acc;
  const int64_t* __restrict__ props = RJ.props;
  const double* __restrict__ X = RJ.X;
  const int d = RJ.d;
  double* __restrict__ Xp = RJ.Xp;
  for (int q = vb * 256 + (int)threadIdx.x; q < s * d; q += vg * 256) {
    const int j = q / d, t = q % d;
    Xp[q] = X[props[acc[j]] * d + t];
  }
}

// Squared distance by direct differences (a point paired with itself gives 0).
__device__ __attribute__((always_inline)) inline double sqdist(const double* __restrict__ x, const double* __restrict__ y, int d) {
  double s = 0.0;
  for (int t = 0; t < d; ++t) {
    const double e = x[t] - y[t];
    s += e * e;
  }
  return s;
}

}  // namespace arpc
