// Accelerated RPCholesky, low-memory implementation (Alg. 3, Section 2.4):
// the kernels and the host code of arpc_factor_lowmem.
//
// No N x k factor is kept.  The state between rounds is the pivot list S,
// their coordinates, the lower Cholesky factor L of A(S,S) (k x k, the
// caller's output) and the residual diagonal u.  A round:
//   1. proposals from u (shared with arpc_factor);
//   2. H = A(S',S') - Y^* Y with Y = L^{-1} A(S,S'): kernel block, forward
//      substitution, a rank-k_r product;
//   3. RejectionSampleSubmatrix (shared), giving S_i and its factor L_i;
//   4. the residual diagonal: with W = L^{-*} L^{-1} A(S,S_i), the new
//      columns are G = (A(:,S_i) - A(:,S) W) L_i^{-*} = A(:, S u S_i) Z for
//      Z = [-W L_i^{-*}; L_i^{-*}], so one pass regenerates each row's
//      kernel values against all pivots, contracts them with Z and keeps
//      only |G(row, :)|^2 (as partial sums over 64-column groups);
//   5. L gains the rows [Y(:,T)^*, L_i].
// Everything is FP64 with direct-difference distances, as in the oracle.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_host.h"
#include "arpc_launch.h"

namespace arpc {
namespace {

constexpr int LM_KMAX = 4096;   // longest solution vector kept in LDS
constexpr int LM_BMAX = 512;    // inverse factor of L_i by linv_column
constexpr int LM_DMAX = 256;    // staged pivot coordinates in the row kernel
constexpr int LM_JC = 16;       // pivots per staged chunk in the row kernel (a multiple of 4)
constexpr int LM_CG = 64;       // columns of G per row-norm partial (the group width k_diag reads)
constexpr int LM_CS = 192;      // columns of G per workgroup in the row kernel (three groups)

typedef double rd4 __attribute__((ext_vector_type(4)));

// Kt(j, c) = kappa(x_{S_j}, x_{S'_c}) for j < k_r, c < b: A(S, S'), column-major (ld ldk).
__global__ __launch_bounds__(256) void k_lm_cross(const double* __restrict__ X, int d, KParams kp,
                                                  const int64_t* __restrict__ props, int b,
                                                  const double* __restrict__ XS, int64_t ldk,
                                                  double* __restrict__ Kt, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int64_t kr = st->k_r;
  const int c = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= b || j >= kr) return;
  Kt[(int64_t)c * ldk + j] = kappa_r2(sqdist(XS + j * d, X + props[c] * d, d), kp);
}

// Forward substitution, column c of B (length k_r, ld ldk) <- L^{-1} column c,
// for c < ncols, one wavefront per column, by 64-row blocks: the rows of block
// J first subtract L(J, <J) y(<J) (loads independent of the chain), then the
// 64 x 64 diagonal block is solved step by step with its column values loaded
// up front (lane i holds L(i, t); lane t holds the diagonal).
__global__ __launch_bounds__(64) void k_lm_fwd(const double* __restrict__ L, int64_t ldl, double* __restrict__ B,
                                               int64_t ldk, int ncols, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int kr = (int)st->k_r;
  const int c = blockIdx.x;
  if (c >= ncols || kr == 0) return;
  __shared__ double y[LM_KMAX];
  const int lane = threadIdx.x;
  double* col = B + (int64_t)c * ldk;
  for (int i = lane; i < kr; i += 64) y[i] = col[i];
  __syncthreads();
  for (int J = 0; 64 * J < kr; ++J) {
    const int i = 64 * J + lane;
    const bool in = i < kr;
    const int ic = in ? i : kr - 1;
    double acc = 0.0;
    for (int t = 0; t < 64 * J; ++t) acc = fma(L[(int64_t)t * ldl + ic], y[t], acc);
    double lv[64];
#pragma unroll
    for (int tt = 0; tt < 64; ++tt) {
      const int t = 64 * J + tt < kr ? 64 * J + tt : kr - 1;
      lv[tt] = L[(int64_t)t * ldl + ic];
    }
    double yi = in ? y[ic] - acc : 0.0;
#pragma unroll
    for (int tt = 0; tt < 64; ++tt) {
      if (64 * J + tt < kr) {
        const double yt = readlane_f64(yi, tt) / readlane_f64(lv[tt], tt);
        yi = lane == tt ? yt : (lane > tt ? fma(-lv[tt], yt, yi) : yi);
      }
    }
    if (in) y[i] = yi;
    __syncthreads();
  }
  for (int i = lane; i < kr; i += 64) col[i] = y[i];
}

// Backward substitution with L^*: column c of W (length k_r) <- L^{-*} column
// c, for c < s_r, by 64-row blocks from the last: block J first subtracts
// L(>J, J)^* w(>J) (lane i walks column i of L, contiguous), then solves its
// diagonal block from the bottom row up (lane i holds L(t, i)).
__global__ __launch_bounds__(64) void k_lm_bwd(const double* __restrict__ L, int64_t ldl, double* __restrict__ W,
                                               int64_t ldk, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int kr = (int)st->k_r, s = st->s_r;
  const int c = blockIdx.x;
  if (c >= s || kr == 0) return;
  __shared__ double w[LM_KMAX];
  const int lane = threadIdx.x;
  double* col = W + (int64_t)c * ldk;
  for (int i = lane; i < kr; i += 64) w[i] = col[i];
  __syncthreads();
  for (int J = (kr + 63) / 64 - 1; J >= 0; --J) {
    const int i = 64 * J + lane;
    const bool in = i < kr;
    const int ic = in ? i : kr - 1;
    const double* li = L + (int64_t)ic * ldl;   // column i of L
    double acc = 0.0;
    for (int t = 64 * (J + 1); t < kr; ++t) acc = fma(li[t], w[t], acc);
    double lv[64];
#pragma unroll
    for (int tt = 0; tt < 64; ++tt) {
      const int t = 64 * J + tt < kr ? 64 * J + tt : kr - 1;
      lv[tt] = li[t];                             // L(t, i)
    }
    double wi = in ? w[ic] - acc : 0.0;
#pragma unroll
    for (int tt = 63; tt >= 0; --tt) {
      if (64 * J + tt < kr) {
        const double wt = readlane_f64(wi, tt) / readlane_f64(lv[tt], tt);
        wi = lane == tt ? wt : (lane < tt ? fma(-lv[tt], wt, wi) : wi);
      }
    }
    if (in) w[i] = wi;
    __syncthreads();
  }
  for (int i = lane; i < kr; i += 64) col[i] = w[i];
}

// H(i, j) -= sum_t Y(t, i) Y(t, j) over t < k_r, in 16 x 16 blocks of H
// with the 32 columns of Y staged through LDS 64 rows at a time.
__global__ __launch_bounds__(256) void k_lm_syrk(double* __restrict__ H, int b, const double* __restrict__ Y,
                                                 int64_t ldk, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int kr = (int)st->k_r;
  if (kr == 0) return;
  __shared__ double ys[2][16][65];
  const int tid = threadIdx.x, ti = tid % 16, tj = tid / 16;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int sd = tid % 64, sr = tid / 64;
  const double* src[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int r = sr + 4 * m;
    const int cc = r < 16 ? i0 + r : j0 + r - 16;
    src[m] = Y + (int64_t)(cc < b ? cc : b - 1) * ldk;
  }
  double sum = 0.0;
  for (int t0 = 0; t0 < kr; t0 += 64) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int r = sr + 4 * m;
      ys[r / 16][r % 16][sd] = t0 + sd < kr ? src[m][t0 + sd] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < 64; ++t) sum = fma(ys[0][ti][t], ys[1][tj][t], sum);
  }
  const int i = i0 + ti, j = j0 + tj;
  if (i < b && j < b) H[(int64_t)j * b + i] -= sum;
}

// For the accepted proposals a < s_r: XS(k_r + a, :) = X(pivot, :), and
// column a of YT and of W = column acc[a] of Y.
__global__ __launch_bounds__(256) void k_lm_take(const double* __restrict__ X, int d,
                                                 const int64_t* __restrict__ pivots, double* __restrict__ XS,
                                                 const double* __restrict__ Y, const int32_t* __restrict__ acc,
                                                 double* __restrict__ YT, double* __restrict__ W, int64_t ldk,
                                                 const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int64_t kr = st->k_r;
  const int a = blockIdx.x;
  if (a >= st->s_r) return;
  const int64_t p = pivots[kr + a];
  for (int t = threadIdx.x; t < d; t += 256) XS[(kr + a) * d + t] = X[p * d + t];
  const double* yc = Y + (int64_t)acc[a] * ldk;
  for (int64_t t = threadIdx.x; t < kr; t += 256) {
    YT[(int64_t)a * ldk + t] = yc[t];
    W[(int64_t)a * ldk + t] = yc[t];
  }
}

// Li = L_i^{-1} (s_r x s_r, column-major ld b), column c by one wavefront.
__global__ __launch_bounds__(64) void k_lm_linv(LFactor Lf, double* __restrict__ Li, int b, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r, c = blockIdx.x, lane = threadIdx.x;
  if (c >= s) return;
  if (s <= 256) {
    double r[4];
    linv_column(Lf, s, c, lane, r);
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (lane + 64 * m < s) Li[(int64_t)c * b + lane + 64 * m] = r[m];
  } else {
    double r[8];
    linv_column(Lf, s, c, lane, r);
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (lane + 64 * m < s) Li[(int64_t)c * b + lane + 64 * m] = r[m];
  }
}

// Z (row j, column c < s_r; row-major, ld b): Z(j, c) = -sum_{c2 <= c}
// W(j, c2) Li(c, c2) for j < k_r, and Z(k_r + a, c) = Li(c, a).
__global__ __launch_bounds__(256) void k_lm_z(const double* __restrict__ W, int64_t ldk,
                                              const double* __restrict__ Li, int b, double* __restrict__ Z,
                                              const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int kr = (int)st->k_r, s = st->s_r;
  const int j = blockIdx.y;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= s || j >= kr + s) return;
  double z;
  if (j < kr) {
    double acc = 0.0;
    for (int c2 = 0; c2 <= c; ++c2) acc = fma(W[(int64_t)c2 * ldk + j], Li[(int64_t)c2 * b + c], acc);
    z = -acc;
  } else {
    const int a = j - kr;
    z = c >= a ? Li[(int64_t)a * b + c] : 0.0;
  }
  Z[(int64_t)j * b + c] = z;
}

// P(g, row) = |G(row, 64 g .. 64 g + 63)|^2, G(row, :) = sum_j kappa(x_row,
// x_{S_j}) Z(j, :) over all k_r + s_r pivots, on the FP64 matrix cores.
// Workgroup (x, y) takes rows 64 x .. 64 x + 63 (16 per wavefront) and the
// LM_CS columns from LM_CS y; the pivots' coordinates and that slice of Z are
// staged through LDS LM_JC pivots at a time, the next chunk's Z (and, for
// d <= 16, coordinates) loaded into registers during the current one.  Per
// step of four pivots, lane (g, l16) evaluates kappa(x_{row l16},
// x_{S_{j + g}}) once, in FP64 with direct differences, and that value is the
// A operand of the slice's 16x16x4 products with Z (B operand: lane (g, l16)
// holds Z(j + g, column l16 of the tile)).  Accumulator entry i of lane (g, l16) is G(row g + 4 i,
// column l16 of the tile); the squares of each 64-column group are summed
// over its four tiles and then across the 16 lanes of a row.  XR: the row's
// coordinates in registers (d <= 16).
template <int XR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_lm_rows(const double* __restrict__ X, int d, KParams kp,
                                                 const double* __restrict__ XS, const double* __restrict__ Z,
                                                 int b, double* __restrict__ P, int64_t N, const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  constexpr int CT = LM_CS / 16;   // column tiles of the slice
  const int s = st->s_r;
  const int kt = (int)st->k_r + s;
  const int c0 = blockIdx.y * LM_CS;
  if (s == 0 || c0 >= s) return;
  __shared__ double xs[LM_JC * LM_DMAX];
  __shared__ double zs[LM_JC][LM_CS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * w;   // this wavefront's 16 rows
  const int64_t myrow = row0 + l16;                          // the row whose kernel values this lane forms
  const double* xrow = X + (myrow < N ? myrow : N - 1) * d;
  double xr[XR > 0 ? XR : 1];
  if constexpr (XR > 0) {
#pragma unroll
    for (int t = 0; t < XR; ++t) xr[t] = t < d ? xrow[t] : 0.0;
  }
  rd4 acc[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) acc[ct] = rd4{0.0, 0.0, 0.0, 0.0};
  const int64_t nxs = (int64_t)kt * d;
  // the next chunk is loaded into registers while the current one is used
  constexpr int ZPT = LM_JC * LM_CS / 256;                // Z values per thread per chunk
  constexpr int XPT = (LM_JC * 16 + 255) / 256;   // coordinates per thread (prefetched when d <= 16)
  double zn[ZPT], xn[XPT];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int r = 0; r < ZPT; ++r) {
      const int e = tid + 256 * r, jj = e / LM_CS, m = e % LM_CS;
      zn[r] = (j0 + jj < kt && c0 + m < s) ? Z[(int64_t)(j0 + jj) * b + c0 + m] : 0.0;
    }
    if constexpr (XR > 0) {
#pragma unroll
      for (int r = 0; r < XPT; ++r) {
        const int e = tid + 256 * r;
        const int64_t q = (int64_t)j0 * d + e;
        xn[r] = (e < LM_JC * d && q < nxs) ? XS[q] : 0.0;
      }
    }
  };
  fetch(0);
  for (int j0 = 0; j0 < kt; j0 += LM_JC) {
    __syncthreads();   // the previous chunk is consumed
#pragma unroll
    for (int r = 0; r < ZPT; ++r) {
      const int e = tid + 256 * r;
      zs[e / LM_CS][e % LM_CS] = zn[r];
    }
    if constexpr (XR > 0) {
#pragma unroll
      for (int r = 0; r < XPT; ++r) {
        const int e = tid + 256 * r;
        if (e < LM_JC * d) xs[e] = xn[r];
      }
    } else {
      for (int e = tid; e < LM_JC * d; e += 256) {
        const int64_t q = (int64_t)j0 * d + e;
        xs[e] = q < nxs ? XS[q] : 0.0;
      }
    }
    __syncthreads();
    if (j0 + LM_JC < kt) fetch(j0 + LM_JC);
    // pivots past kt have zero rows of Z (their coordinates are staged as 0,
    // so their kernel values are finite).  Each step's kernel value is
    // formed one step ahead, so its arithmetic runs beside the previous
    // step's products instead of in front of its own.
    auto kval = [&](int q) __attribute__((always_inline)) {
      const double* xp = xs + (4 * q + g) * d;
      double r2 = 0.0;
      if constexpr (XR > 0) {
#pragma unroll
        for (int t = 0; t < XR; ++t)
          if (t < d) {
            const double e = xr[t] - xp[t];
            r2 += e * e;
          }
      } else {
        for (int t = 0; t < d; ++t) {
          const double e = xrow[t] - xp[t];
          r2 += e * e;
        }
      }
      return kappa_r2(r2, kp);
    };
    double kv = kval(0);
#pragma unroll
    for (int q = 0; q < LM_JC / 4; ++q) {
      const double kvn = q + 1 < LM_JC / 4 ? kval(q + 1) : 0.0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, zs[4 * q + g][16 * ct + l16], acc[ct], 0, 0, 0);
      kv = kvn;
    }
  }
  // |G(row, group)|^2 for the slice's 64-column groups
  const int ng = (s + 63) / 64;
#pragma unroll
  for (int pg = 0; pg < LM_CS / 64; ++pg) {
    const int gi = c0 / 64 + pg;   // group index in P
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double v = 0.0;
#pragma unroll
      for (int ct = 4 * pg; ct < 4 * pg + 4; ++ct) v = fma(acc[ct][i], acc[ct][i], v);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
      const int64_t row = row0 + g + 4 * i;
      if (l16 == 0 && gi < ng && row < N) P[(int64_t)gi * N + row] = v;
    }
  }
}

// Rows k_r + a of L (a < s_r): L(k_r + a, t) = YT(t, a) for t < k_r, and
// L(k_r + a, k_r + c) = L_i(a, c) for c <= a (the rest of the row stays 0).
__global__ __launch_bounds__(256) void k_lm_append_l(double* __restrict__ L, int64_t ldl,
                                                     const double* __restrict__ YT, int64_t ldk, LFactor Lf,
                                                     const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int kr = (int)st->k_r, s = st->s_r;
  const int a = blockIdx.y;
  if (a >= s) return;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < kr + s; t += gridDim.x * 256) {
    const double v = t < kr ? YT[(int64_t)a * ldk + t] : (t - kr <= a ? Lf.at(a, t - kr) : 0.0);
    L[(int64_t)t * ldl + kr + a] = v;
  }
}

// ------------------------------------------------------------ host code
inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct LmLayout {
  size_t st, u, csum, cpre, props, acc, hist, XS, Kt, YT, W, H, Li, Z, P, trace, total;
};

LmLayout lm_layout(const arpc_problem& p) {
  LmLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  };
  const int64_t nch = (p.N + CHUNK - 1) / CHUNK;
  const size_t kb = sizeof(double) * (size_t)p.k * (size_t)p.b;
  l.st = take(sizeof(RoundState));
  l.u = take(sizeof(double) * p.N);
  l.csum = take(sizeof(double) * nch);
  l.cpre = take(sizeof(double) * nch);
  l.props = take(sizeof(int64_t) * p.b);
  l.acc = take(sizeof(int32_t) * p.b);
  l.hist = take(sizeof(int32_t) * (p.k + 1));
  l.XS = take(sizeof(double) * p.k * p.d);
  l.Kt = take(kb);
  l.YT = take(kb);
  l.W = take(kb);
  l.H = take(sizeof(double) * p.b * p.b);
  l.Li = take(sizeof(double) * p.b * p.b);
  l.Z = take(sizeof(double) * (p.k + p.b) * p.b);
  l.P = take(sizeof(double) * ((p.b + LM_CG - 1) / LM_CG) * p.N);
  l.trace = take(sizeof(double));
  l.total = off;
  return l;
}

arpc_status lm_validate(const arpc_problem* p) {
  const arpc_status v = validate(p);
  if (v != ARPC_OK) return v;
  if (p->prec != ARPC_FP64 || p->method != ARPC_ACCEL) return ARPC_EINVAL;
  if (p->k > LM_KMAX || p->b > LM_BMAX || p->d > LM_DMAX) return ARPC_EINVAL;
  return ARPC_OK;
}

void lm_round(hipStream_t s, const arpc_problem& p, const KParams& kp, const Unif& un, char* ws,
              const LmLayout& l, const double* X, double* L, int64_t* pivots, Profiler& prof) {
  const int b = (int)p.b, d = (int)p.d;
  const int64_t N = p.N, k = p.k, nch = (N + CHUNK - 1) / CHUNK;
  RoundState* st = (RoundState*)(ws + l.st);
  double* u = (double*)(ws + l.u);
  double* csum = (double*)(ws + l.csum);
  int64_t* props = (int64_t*)(ws + l.props);
  int32_t* acc = (int32_t*)(ws + l.acc);
  double* XS = (double*)(ws + l.XS);
  double* Kt = (double*)(ws + l.Kt);
  double* YT = (double*)(ws + l.YT);
  double* W = (double*)(ws + l.W);
  double* H = (double*)(ws + l.H);
  double* Li = (double*)(ws + l.Li);
  double* Z = (double*)(ws + l.Z);
  double* P = (double*)(ws + l.P);
  const LFactor Lf{H, acc, b};
  prof.begin(ARPC_KC_PROPOSE);
  launch_propose(s, u, csum, (double*)(ws + l.cpre), nch, N, b, un, st, props);
  prof.end();
  prof.begin(ARPC_KC_GATHER);
  launch_kernel_block(s, X, d, kp, props, b, H, st);
  hipLaunchKernelGGL(k_lm_cross, dim3((unsigned)((k + 255) / 256), (unsigned)b), dim3(256), 0, s, X, d, kp, props, b,
                     XS, k, Kt, st);
  hipLaunchKernelGGL(k_lm_fwd, dim3((unsigned)b), dim3(64), 0, s, L, k, Kt, k, b, st);
  hipLaunchKernelGGL(k_lm_syrk, dim3((unsigned)((b + 15) / 16), (unsigned)((b + 15) / 16)), dim3(256), 0, s, H, b,
                     Kt, k, st);
  prof.end();
  prof.begin(ARPC_KC_REJECT);
  launch_reject(s, H, b, props, un, st, acc, pivots, u, k, false);
  prof.end();
  prof.begin(ARPC_KC_PREP);
  hipLaunchKernelGGL(k_lm_take, dim3((unsigned)b), dim3(256), 0, s, X, d, pivots, XS, Kt, acc, YT, W, k, st);
  hipLaunchKernelGGL(k_lm_bwd, dim3((unsigned)b), dim3(64), 0, s, L, k, W, k, st);
  hipLaunchKernelGGL(k_lm_linv, dim3((unsigned)b), dim3(64), 0, s, Lf, Li, b, st);
  hipLaunchKernelGGL(k_lm_z, dim3((unsigned)((b + 255) / 256), (unsigned)(k + b)), dim3(256), 0, s, W, k, Li, b, Z,
                     st);
  prof.end();
  prof.begin(ARPC_KC_COLGEMM);
  const dim3 grows((unsigned)((N + 63) / 64), (unsigned)((b + LM_CS - 1) / LM_CS));
  if (d <= 16)
    if (d <= 8) hipLaunchKernelGGL(k_lm_rows<8>, grows, dim3(256), 0, s, X, d, kp, XS, Z, b, P, N, st);
    else hipLaunchKernelGGL(k_lm_rows<16>, grows, dim3(256), 0, s, X, d, kp, XS, Z, b, P, N, st);
  else
    hipLaunchKernelGGL(k_lm_rows<0>, grows, dim3(256), 0, s, X, d, kp, XS, Z, b, P, N, st);
  prof.end();
  prof.begin(ARPC_KC_DIAG);
  launch_diag(s, u, csum, P, LM_CG, N, nch, st);
  prof.end();
  prof.begin(ARPC_KC_FINISH);
  hipLaunchKernelGGL(k_lm_append_l, dim3((unsigned)((k + b + 255) / 256 < 16 ? (k + b + 255) / 256 : 16), (unsigned)b),
                     dim3(256), 0, s, L, k, YT, k, Lf, st);
  launch_finish(s, st, b, k, p.max_rounds, (int32_t*)(ws + l.hist));
  prof.end();
}

#define LMCHK(x)                              \
  do {                                        \
    if ((x) != hipSuccess) return ARPC_EDEVICE; \
  } while (0)

arpc_status lm_run(const arpc_problem& p, const double* X, double* L, int64_t* pivots, char* ws, const LmLayout& l,
                   hipStream_t s, arpc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  Profiler prof(s, g_profiling);
  const KParams kp = kparams_of(p);
  const Unif un{nullptr, 0, p.seed};
  const int64_t nch = (p.N + CHUNK - 1) / CHUNK;
  RoundState* st = (RoundState*)(ws + l.st);
  LMCHK(hipMemsetAsync(st, 0, sizeof(RoundState), s));
  LMCHK(hipMemsetAsync(L, 0, sizeof(double) * (size_t)p.k * (size_t)p.k, s));
  prof.begin(ARPC_KC_INIT);
  launch_init(s, (double*)(ws + l.u), (double*)(ws + l.csum), X, p.N, (int)p.d, kp, st, nch);
  prof.end();
  LMCHK(hipGetLastError());
  RoundState h{};
  int64_t known_k = 0, enqueued = 0;
  for (;;) {
    int64_t batch = (p.k - known_k + p.b - 1) / p.b;
    if (batch < 1) batch = 1;
    if (p.max_rounds > 0 && enqueued + batch > p.max_rounds) batch = p.max_rounds - enqueued;
    if (batch < 1) batch = 1;
    for (int64_t r = 0; r < batch; ++r) lm_round(s, p, kp, un, ws, l, X, L, pivots, prof);
    enqueued += batch;
    LMCHK(hipGetLastError());
    LMCHK(hipMemcpyAsync(&h, st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    LMCHK(hipStreamSynchronize(s));
    prof.collect();
    if (h.status != ST_RUNNING) break;
    known_k = h.k_r;
  }
  if (h.nonfinite) return ARPC_ENUMERIC;
  if (h.status == ST_NOUNIF) return ARPC_EINVAL;
  double* tr = (double*)(ws + l.trace);
  launch_trace(s, (double*)(ws + l.csum), nch, tr);
  double trace_resid = 0.0;
  LMCHK(hipMemcpyAsync(&trace_resid, tr, sizeof(double), hipMemcpyDeviceToHost, s));
  const int64_t k_out = h.k_r;
  if (k_out < p.k) LMCHK(hipMemsetAsync(pivots + k_out, 0xff, sizeof(int64_t) * (size_t)(p.k - k_out), s));
  LMCHK(hipStreamSynchronize(s));
  const arpc_status ret =
      (k_out == p.k || (p.max_rounds > 0 && h.round >= p.max_rounds && h.status == ST_DONE)) ? ARPC_OK
                                                                                           : ARPC_EARLY_STOP;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->k_out = k_out;
    stats->rounds = h.round;
    stats->proposals = h.proposals;
    stats->status = ret;
    stats->trace_A = h.trace_A;
    stats->trace_resid = trace_resid;
    for (int c = 0; c < ARPC_NUM_KC; ++c) {
      stats->ms_kernel[c] = prof.ms[c];
      stats->launches[c] = prof.n[c];
    }
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return ret;
}

}  // namespace
}  // namespace arpc

using namespace arpc;

extern "C" {

arpc_status arpc_lowmem_workspace_size(const arpc_problem* problem, size_t* bytes) {
  const arpc_status v = lm_validate(problem);
  if (v != ARPC_OK) return v;
  if (!bytes) return ARPC_EINVAL;
  *bytes = lm_layout(*problem).total;
  return ARPC_OK;
}

arpc_status arpc_factor_lowmem(const arpc_problem* problem, const double* X, double* L, int64_t* pivots, void* ws,
                               size_t ws_bytes, void* stream, arpc_stats* stats) {
  const arpc_status v = lm_validate(problem);
  if (v != ARPC_OK) return v;
  if (!X || !L || !pivots || !ws) return ARPC_EINVAL;
  if (((uintptr_t)X & 7) || ((uintptr_t)L & 7) || ((uintptr_t)pivots & 7) || ((uintptr_t)ws & 255))
    return ARPC_EINVAL;
  const LmLayout l = lm_layout(*problem);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  return lm_run(*problem, X, L, pivots, (char*)ws, l, (hipStream_t)stream, stats);
}

}  // extern "C"
