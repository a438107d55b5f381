// HIP kernels of the per-step stress evaluation and friction update (gfx950).
//
// One predictor-corrector step (Section 2.4) on one stream:
//   k_hmat        interaction history part (lags >= 1 and the static tail): every
//                 work item (a run of lags of one H-matrix block) streams its
//                 factors once, with the slip-rate history rows of its lags staged
//                 in LDS; S partial sums per receiver row (S time windows)
//   k_hmat_mfma16 the same for FP32 factors and S = 16 on the matrix cores
//                 (16-bit factors: kernels_x16.hip)
//   k_reduce_*    fixed-order sums of each receiver's partials, times -mu/(2cs)
//   k_self_hist   per-mode time convolution over lags T >= 1 (ragged windows)
//   k_dft         explicit transform of the predicted / corrected slip, modal stress
//   k_stage       inverse transform per element, Newton solve in ln V, state
//                 update; the corrector commits the step and appends the histories
// Every reduction has a fixed order (no floating-point atomics).
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace seas {


// ------------------------------------------------------------------ H-matrix apply
// One work item per workgroup: a run of consecutive lags T_first .. T_first+nl-1
// of one block (factors contiguous in the arena) applied to S consecutive history
// windows: window k of lag T reads the rate row of time head + k - T. The item's
// rows span nl + S - 1 consecutive times and are staged in LDS once, newest
// first: row rho holds time head + S - 1 - T_first - rho, so lag l, window k is
// row l + S - 1 - k, and for the dense inner index e = l*q + j the value is
// h[e + (S-1-k) q].
//   low rank: z[c][k] = w_c . h(lag(c), k), then y[i][k] = sum_c U[c][i] z[c][k]
//   dense:    y[i][k] = sum_{l,j} D_l[i][j] h(l, k)[j]
// Rows are processed by G = 256/p groups of p threads (coalesced factor reads),
// each over a contiguous range of the inner index; group partials are added in
// group order. Output: S partial sums per row at out[i * pstride + k].

// acc[k] += sum over e in [e0, e1) of M[e*p + i] * x(e, k); 8 factor loads are
// issued before their multiply-adds so that enough bytes are in flight per CU.
template <typename TF, typename TA, int S, typename X>
__device__ __forceinline__ void accum_rows(const TF* __restrict__ M, int p, int i, int e0, int e1, X x,
                                           TA (&acc)[S]) {
  const TF* m = M + (int64_t)e0 * p + i;
  int e = e0;
  for (; e + 8 <= e1; e += 8, m += 8 * p) {
    TA mv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) mv[u] = (TA)m[u * p];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < S; ++k) acc[k] += mv[u] * x(e + u, k);
    }
  }
  for (; e < e1; ++e, m += p) {
    const TA m0 = (TA)m[0];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] += m0 * x(e, k);
  }
}

template <typename TF, typename TA, int S, typename X>
__device__ __forceinline__ void rows_apply(const TF* __restrict__ M, int E, int p, X x, TA* red,
                                           double* __restrict__ out, int pstride) {
  const int tid = threadIdx.x;
  if (p <= kItemThreads) {
    const int G = kItemThreads / p;
    const int g = tid / p, i = tid - g * p;
    TA acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0;
    if (g < G) {
      const int e0 = (int)((int64_t)E * g / G), e1 = (int)((int64_t)E * (g + 1) / G);
      accum_rows<TF, TA, S>(M, p, i, e0, e1, x, acc);
    }
    __syncthreads();  // red aliases the staged history
    if (g < G) {
#pragma unroll
      for (int k = 0; k < S; ++k) red[(g * p + i) * S + k] = acc[k];
    }
    __syncthreads();
    for (int e = tid; e < p * S; e += kItemThreads) {
      const int ii = e / S, k = e - ii * S;
      TA s = 0;
      for (int gg = 0; gg < G; ++gg) s += red[(gg * p + ii) * S + k];
      out[ii * pstride + k] = (double)s;
    }
  } else {
    for (int i = tid; i < p; i += kItemThreads) {
      TA acc[S];
#pragma unroll
      for (int k = 0; k < S; ++k) acc[k] = 0;
      accum_rows<TF, TA, S>(M, p, i, 0, E, x, acc);
#pragma unroll
      for (int k = 0; k < S; ++k) out[i * pstride + k] = (double)acc[k];
    }
  }
}

template <typename TF, typename TA, int S>
__global__ __launch_bounds__(kItemThreads) void k_hmat(const Item* __restrict__ items, const int32_t* __restrict__ lagT,
                                                       const int32_t* __restrict__ lagCol,
                                                       const int32_t* __restrict__ lagColOff,
                                                       const TF* __restrict__ arena, const TF* __restrict__ ring,
                                                       int64_t head, int64_t R, int N,
                                                       const double* __restrict__ tail_acc,
                                                       double* __restrict__ partials, int pstride,
                                                       const int64_t* __restrict__ clk) {
  if (clk) head += *clk;
  __shared__ TA h[kHistMax];
  __shared__ TA z[kZMax];
  __shared__ int cl[kColMax];  // lag index of each low-rank column
  const Item it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int q = it.q, p = it.p, nl = it.nlag;
  if (it.src == 0) {
    const int span = nl + S - 1;
    const int64_t tnew = head + S - 1 - lagT[it.lag_off];
    for (int e = tid; e < span * q; e += kItemThreads) {
      const int r = e / q, j = e - r * q;
      h[e] = (TA)ring[ring_slot(tnew - r, R) * N + it.col0 + j];
    }
  } else {  // static tail: one row, the pair's expired slip (S = 1)
    for (int j = tid; j < q; j += kItemThreads) h[j] = (TA)tail_acc[it.tail_off + j];
  }
  double* out = partials + it.part;
  const TF* base = arena + it.data;
  if (it.kind == 0) {
    const int nc = it.ncol;
    const int32_t* cp = lagCol + lagColOff[blockIdx.x];
    for (int l = 0; l < nl; ++l)
      for (int c = cp[l] + tid; c < cp[l + 1]; c += kItemThreads) cl[c] = l;
    __syncthreads();
    // projection, one thread per column; W panel [q][nc]
    for (int c = tid; c < nc; c += kItemThreads) {
      const TA* hc = h + (cl[c] + S - 1) * q;  // window k is hc - k q
      const TF* w = base + c;
      TA acc[S];
#pragma unroll
      for (int k = 0; k < S; ++k) acc[k] = 0;
      for (int j = 0; j < q; ++j) {
        const TA wv = (TA)w[(int64_t)j * nc];
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] += wv * hc[j - k * q];
      }
#pragma unroll
      for (int k = 0; k < S; ++k) z[c * S + k] = acc[k];
    }
    __syncthreads();
    // expansion y = U z; U panel [nc][p]
    rows_apply<TF, TA, S>(base + (int64_t)q * nc, nc, p, [&](int c, int k) { return z[c * S + k]; }, h, out,
                          pstride);
  } else {
    __syncthreads();
    // inner index e = l*q + j over [nlag][q][p]
    rows_apply<TF, TA, S>(base, nl * q, p, [&](int e, int k) { return h[e + (S - 1 - k) * q]; }, h, out,
                          pstride);
  }
}

// ------------------------------------------------------------------ MFMA form
// FP32 factors with S = 16 windows: every item is a skinny GEMM with N = 16
// (the windows), run on the matrix cores with v_mfma_f32_16x16x4_f32. For one
// 16x16 output tile and 4 consecutive inner indices e:
//   A operand (16 rows x 4): lane l holds A[row l%16][e + l/16]
//   B operand (4 x 16):      lane l holds B[e + l/16][window l%16]
//   accumulator: lane l, register v holds Y[row 4 (l/16) + v][window l%16]
// so a factor element is read once from HBM and used 16 times, and the history
// comes from LDS once per 16 multiply-adds.

template <typename FA, typename FB>
__device__ __forceinline__ mfma_f4 mfma_run(int e0, int e1, FA A, FB B, mfma_f4 acc, int lane) {
  const int sub = lane >> 4, col = lane & 15;
  for (int e = e0; e < e1; e += 16) {  // 4 steps of 4, operands loaded first
    float a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ee = e + 4 * u + sub;
      const bool ok = ee < e1;
      a[u] = ok ? A(ee, col) : 0.0f;
      b[u] = ok ? B(ee, col) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
  }
  return acc;
}

// One super-tile of TW consecutive 16-row tiles (rows t0*16 ..) over the inner
// range [e0, e1): the operands of 4 inner steps (TW factor loads + 1 history load
// each) are issued before their MFMAs so that enough bytes are in flight.
template <int TW, typename FB>
__device__ __forceinline__ void mfma_supertile(const float* __restrict__ M, int p, int t0, int e0, int e1, FB B,
                                               mfma_f4 (&acc)[TW], int lane) {
  constexpr int PF = TW <= 4 ? 4 : 2;  // inner steps whose operands are loaded ahead
  const int sub = lane >> 4, col = lane & 15;
#pragma unroll
  for (int u = 0; u < TW; ++u) acc[u] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int e = e0; e < e1; e += 4 * PF) {
    float a[PF][TW], b[PF];
#pragma unroll
    for (int w4 = 0; w4 < PF; ++w4) {
      const int ee = e + 4 * w4 + sub;
      const bool ok = ee < e1;
      b[w4] = ok ? B(ee, col) : 0.0f;
      const float* row = M + (int64_t)ee * p + t0 * 16 + col;
#pragma unroll
      for (int u = 0; u < TW; ++u) a[w4][u] = (ok && (t0 + u) * 16 + col < p) ? row[u * 16] : 0.0f;
    }
#pragma unroll
    for (int w4 = 0; w4 < PF; ++w4) {
#pragma unroll
      for (int u = 0; u < TW; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[w4][u], b[w4], acc[u], 0, 0, 0);
    }
  }
}

template <int TW>
__device__ __forceinline__ void mfma_store(const mfma_f4 (&acc)[TW], int p, int t0, float* __restrict__ out,
                                           int pstride, int lane) {
#pragma unroll
  for (int u = 0; u < TW; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = (t0 + u) * 16 + 4 * (lane >> 4) + v;
      if (i < p) out[i * pstride + (lane & 15)] = acc[u][v];
    }
  }
}

// Y (p x 16) = sum_e M[e*p + i] B(e, k), e in [0, E), on the matrix cores.
// Small blocks (at most 3 row tiles of 16): the 4 waves take a quarter of the
// inner range each over all row tiles, and their partial tiles are added in wave
// order through LDS (red, which aliases the staged history, needs 3072 floats).
// Larger blocks: each wave takes super-tiles of up to 8 consecutive row tiles
// over the whole inner range, so one B fragment feeds up to 8 MFMAs and the
// factor loads of consecutive tiles are contiguous.
template <typename FB>
__device__ __forceinline__ void mfma_rows(const float* __restrict__ M, int E, int p, FB B, float* red,
                                          float* __restrict__ out, int pstride) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int RT = (p + 15) >> 4;
  if (RT <= 3) {
    const int e0 = ((int)((int64_t)E * wave / 4)) & ~3;
    const int e1 = wave == 3 ? E : (((int)((int64_t)E * (wave + 1) / 4)) & ~3);
    float part[3][4] = {};
    if (RT == 1) {
      mfma_f4 acc[1];
      mfma_supertile<1>(M, p, 0, e0, e1, B, acc, lane);
      for (int v = 0; v < 4; ++v) part[0][v] = acc[0][v];
    } else if (RT == 2) {
      mfma_f4 acc[2];
      mfma_supertile<2>(M, p, 0, e0, e1, B, acc, lane);
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 4; ++v) part[u][v] = acc[u][v];
    } else {
      mfma_f4 acc[3];
      mfma_supertile<3>(M, p, 0, e0, e1, B, acc, lane);
      for (int u = 0; u < 3; ++u)
        for (int v = 0; v < 4; ++v) part[u][v] = acc[u][v];
    }
    __syncthreads();  // every wave is done with the history that red aliases
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      if (u < RT) {
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 3 + u) * 256 + lane * 4 + v] = part[u][v];
      }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < RT * 256; x += kItemThreads) {
      const int u = x >> 8, w = x & 255, ln = w >> 2, v = w & 3;
      float sum = 0.0f;
      for (int wv = 0; wv < 4; ++wv) sum += red[(wv * 3 + u) * 256 + ln * 4 + v];
      const int i = u * 16 + 4 * (ln >> 4) + v;
      if (i < p) out[i * pstride + (ln & 15)] = sum;
    }
    return;
  }
  const int TW = min(8, (RT + 3) / 4);
  const int NST = (RT + TW - 1) / TW;
  for (int st = wave; st < NST; st += 4) {
    const int t0 = st * TW, tw = min(TW, RT - t0);
#define SEAS_TW_CASE(n)                                      \
  case n: {                                                  \
    mfma_f4 acc[n];                                          \
    mfma_supertile<n>(M, p, t0, 0, E, B, acc, lane);         \
    mfma_store<n>(acc, p, t0, out, pstride, lane);           \
  } break;
    switch (tw) {
      SEAS_TW_CASE(1)
      SEAS_TW_CASE(2)
      SEAS_TW_CASE(3)
      SEAS_TW_CASE(4)
      SEAS_TW_CASE(5)
      SEAS_TW_CASE(6)
      SEAS_TW_CASE(7)
      SEAS_TW_CASE(8)
      default: break;
    }
#undef SEAS_TW_CASE
  }
}

__global__ __launch_bounds__(kItemThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_hmat_mfma16(const Item* __restrict__ items,
                                                              const int32_t* __restrict__ lagT,
                                                              const int32_t* __restrict__ lagCol,
                                                              const int32_t* __restrict__ lagColOff,
                                                              const float* __restrict__ arena,
                                                              const float* __restrict__ ring, int64_t head,
                                                              int64_t R, int N, float* __restrict__ partials,
                                                              int pstride, const int64_t* __restrict__ clk) {
  if (clk) head += *clk;
  constexpr int S = 16;
  __shared__ float h[kHistMax];
  __shared__ float z[kZMax];
  const Item it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = it.q, p = it.p, nl = it.nlag;
  {
    const int span = nl + S - 1;
    const int64_t tnew = head + S - 1 - lagT[it.lag_off];
    for (int e = tid; e < span * q; e += kItemThreads) {
      const int r = e / q, j = e - r * q;
      h[e] = ring[ring_slot(tnew - r, R) * N + it.col0 + j];
    }
  }
  float* out = partials + it.part;
  const float* base = arena + it.data;
  __syncthreads();
  if (it.kind == 0) {
    const int nc = it.ncol;
    const int32_t* cp = lagCol + lagColOff[blockIdx.x];
    // projection per lag: Z_l (k_l x 16) = W_l^T H_l, column tiles of 16 spread over waves
    int tile = 0;
    for (int l = 0; l < nl; ++l) {
      const int cb = cp[l], ce = cp[l + 1];
      for (int c0 = cb; c0 < ce; c0 += 16, ++tile) {
        if ((tile & 3) != wave) continue;
        const float* hl = h + (l + S - 1) * q;  // window k is hl - k q
        mfma_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mfma_run(0, q,
                       [&](int j, int c) { const int cc = c0 + c; return cc < ce ? base[(int64_t)j * nc + cc] : 0.0f; },
                       [&](int j, int k) { return hl[j - k * q]; }, acc, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cc = c0 + 4 * (lane >> 4) + v;
          if (cc < ce) z[cc * S + (lane & 15)] = acc[v];
        }
      }
    }
    __syncthreads();
    mfma_rows(base + (int64_t)q * nc, nc, p, [&](int c, int k) { return z[c * S + k]; }, h, out, pstride);
  } else {
    mfma_rows(base, nl * q, p, [&](int e, int k) { return h[e + (S - 1 - k) * q]; }, h, out, pstride);
  }
}

// One 64-lane wave per receiver: lanes stride over the receiver's partial list,
// then a butterfly sum (fixed order, independent of scheduling).
// Far partials: S values per (item, row); f_far[k*N + r] = -eta sum.
template <int S, typename TP>
__global__ void k_reduce_far(const TP* __restrict__ partials, const int32_t* __restrict__ ptr,
                             const int32_t* __restrict__ idx, int N, double neg_eta, double* __restrict__ f) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= N) return;
  double s[S];
#pragma unroll
  for (int k = 0; k < S; ++k) s[k] = 0.0;
  for (int e = ptr[r] + lane; e < ptr[r + 1]; e += 64) {
    const TP* pp = partials + idx[e];
#pragma unroll
    for (int k = 0; k < S; ++k) s[k] += (double)pp[k];
  }
#pragma unroll
  for (int k = 0; k < S; ++k) {
    double v = s[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) f[(int64_t)k * N + r] = neg_eta * v;
  }
}

// Near partials (one per row): f[r] = -eta sum + base[r].
__global__ void k_reduce_near(const double* __restrict__ partials, const int32_t* __restrict__ ptr,
                              const int32_t* __restrict__ idx, int N, double neg_eta,
                              const double* __restrict__ base, double* __restrict__ f) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= N) return;
  double s = 0.0;
  for (int e = ptr[r] + lane; e < ptr[r + 1]; e += 64) s += partials[idx[e]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) f[r] = neg_eta * s + base[r];
}

// ------------------------------------------------------------------ self term
// One 64-lane wave per mode: Fh_n = sum_{T=1}^{W_n} K_n^T D_n^{time0 - T}, where
// time0 is the time of the coefficient being formed; butterfly sum over lanes.
__global__ void k_self_hist(const SelfMode* __restrict__ modes, int n_modes, int nv, int64_t dring_len,
                            const double* __restrict__ tab, const double2* __restrict__ dring, int64_t time0,
                            double2* __restrict__ Fh, const int64_t* __restrict__ clk) {
  if (clk) time0 += *clk;
  const int lane = threadIdx.x & 63;
  const int gg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (gg >= n_modes * nv) return;
  const int v = gg / n_modes, gm = gg - v * n_modes;
  dring += v * dring_len;
  Fh += (int64_t)v * n_modes;
  const SelfMode md = modes[gm];
  double re = 0.0, im = 0.0;
  for (int T = 1 + lane; T <= md.W; T += 64) {
    const double k = tab[md.tab + T];
    const double2 d = dring[md.ring + ring_slot(time0 - T, md.W)];
    re += k * d.x;
    im += k * d.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  if (lane == 0) Fh[gm] = make_double2(re, im);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;  // every lane holds the total (fixed butterfly order)
}

// One 64-lane wave per mode: D_n = sum_j x_j e^{-2 pi i n j / M}, x = delta + coef
// vel (vel may be null), lanes strided over j; F_n = -cfac n (K_n^0 D_n + Fh_n).
// Optionally D_n is stored in the mode's ring at push_time, which must lie in
// the window (ring_head - W_n, ring_head] of the ring's newest time ring_head
// (older times would overwrite newer slots).
__global__ void k_dft(const SelfMode* __restrict__ modes, int n_modes, int nv, int N, int64_t dring_len,
                      const SelfFaultDev* __restrict__ sf, const double* __restrict__ delta,
                      const double* __restrict__ vel, double coef, const double2* __restrict__ tw,
                      const double* __restrict__ tab, const double2* __restrict__ Fh, double2* __restrict__ Fout,
                      double2* __restrict__ dring, int push, int64_t push_time, int64_t ring_head,
                      double2* __restrict__ Dsave, const int64_t* __restrict__ clk) {
  if (clk) {
    push_time += *clk;
    ring_head += *clk;
  }
  const int lane = threadIdx.x & 63;
  const int gg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (gg >= n_modes * nv) return;
  const int v = gg / n_modes, gm = gg - v * n_modes;
  delta += (int64_t)v * N;
  if (vel) vel += (int64_t)v * N;
  if (Fh) Fh += (int64_t)v * n_modes;
  Fout += (int64_t)v * n_modes;
  dring += v * dring_len;
  const SelfMode md = modes[gm];
  const SelfFaultDev f = sf[md.fault];
  const double2* w = tw + f.tw;
  double re = 0.0, im = 0.0;
  for (int j = lane; j < f.Np; j += 64) {
    const double x = vel ? delta[f.off + j] + coef * vel[f.off + j] : delta[f.off + j];
    const double2 e = w[(int)(((int64_t)md.n * j) % f.M)];
    re += x * e.x;
    im += x * e.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane != 0) return;
  const double k0 = tab[md.tab];
  const double c = -f.cfac * md.n;
  const double2 fh = Fh ? Fh[gm] : make_double2(0.0, 0.0);
  Fout[gm] = make_double2(c * (k0 * re + fh.x), c * (k0 * im + fh.y));
  if (push && md.W > 0 && push_time > ring_head - md.W)
    dring[md.ring + ring_slot(push_time, md.W)] = make_double2(re, im);
  if (Dsave) Dsave[(int64_t)v * n_modes + gm] = make_double2(re, im);
}

// Inverse transform at element j, by one wave (lanes strided over modes):
// f_j = (1/M) [2 Re sum_{n=1}^{N_p-1} F_n e^{+2 pi i n j/M} + Re F_{N_p} (-1)^j]  (F_0 = 0)
__device__ __forceinline__ double idft_wave(const SelfFaultDev& f, const double2* __restrict__ F,
                                            const double2* __restrict__ w, int j, int lane) {
  double s = 0.0;
  const int ntop = f.nm < f.Np ? f.nm : f.Np - 1;
  for (int n = 1 + lane; n <= ntop; n += 64) {
    const double2 e = w[(int)(((int64_t)n * j) % f.M)];  // e^{-i...}: Re(F e^{+i...}) = F.x e.x + F.y e.y
    const double2 Fn = F[n - 1];
    s += Fn.x * e.x + Fn.y * e.y;
  }
  s = 2.0 * wave_sum(s);
  if (f.nm >= f.Np) s += F[f.Np - 1].x * ((j & 1) ? -1.0 : 1.0);
  return s / f.M;
}

__device__ __forceinline__ double lag0_apply(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                             const double* __restrict__ val, const double* __restrict__ x, int r) {
  double s = 0.0;
  for (int k = ptr[r]; k < ptr[r + 1]; ++k) s += val[k] * x[col[k]];
  return s;
}

__device__ __forceinline__ double state_rate(double V, double th, double Dc, double eps) {
  const double r = V * th / Dc;
  if (eps == 1.0) return 1.0 - r;
  return (pow(r, -eps) - 1.0) * r / eps;
}

// State after dt at a constant slip rate V: with u = (V theta/Dc)^eps the state
// law reads du/dt = (V/Dc)(1 - u), so u(dt) = u0 e^-x + (1 - e^-x), x = V dt/Dc,
// theta = (Dc/V) u^(1/eps); 1 - e^-x as -expm1(-x) keeps a locked element's state.
__device__ __forceinline__ double state_after(double th0, double V, double Dc, double dt, double eps) {
  const double x = V * dt / Dc;
  const double e = exp(-x), om = -expm1(-x);
  if (eps == 1.0) return th0 * e + Dc / V * om;
  const double u0 = pow(V * th0 / Dc, eps);
  return Dc / V * pow(u0 * e + om, 1.0 / eps);
}

// Newton on x = ln V for A - eta V = sigma_n [f0 + a (x - ln V0) + b ln(V0 theta / Dc)]:
// the residual g is decreasing and concave, so a downward step (taken from the
// right of the root) never crosses it and is taken whole; an upward step longer
// than 1 (g > 0, where A - c - sn a x > eta e^x > 0) stops at
// ln((A - c - sn a x)/eta), above which the root cannot lie, but moves at least 1
// (near the root that bound is lost to cancellation and the steps are short);
// x stays >= -690 (V >= ~1e-300, a rate that is zero
// for every purpose). Stop at |dx| <= 1e-14 max(1, |x|), at most 50 iterations; a
// non-finite iterate fails the solve.
__device__ double newton_lnV(double A, double th, double eta, double a, double b, double Dc, double sn, double V0,
                             double f0, double x, int* fail) {
  constexpr double kXMin = -690.0;
  const double c = sn * (f0 - a * log(V0) + b * log(V0 * th / Dc));
  x = fmax(x, kXMin);
  for (int it = 0; it < 50; ++it) {
    const double ex = exp(x);
    const double g = A - eta * ex - c - sn * a * x;
    if (!isfinite(g)) break;  // (fmax below would hide a NaN)
    const double dg = -eta * ex - sn * a;
    const double step = -g / dg;
    const double up = step > 1.0 ? fmin(step, fmax(log(fmax(A - c - sn * a * x, 1e-300) / eta) - x, 1.0)) : step;
    const double xn = step > 0.0 ? x + up : fmax(x + step, kXMin);
    const double dx = xn - x;
    x = xn;
    if (!(fabs(dx) > 1e-14 * fmax(1.0, fabs(x)))) {
      if (isfinite(x)) return exp(x);
      break;  // a non-finite force balance (e.g. a non-finite stress) fails the solve
    }
  }
  *fail = 1;
  return exp(x);
}

// Expired-slip accumulators that source element r feeds (one per pair, or per
// block with cluster-level windows): E += dt V^t, t = tn - T_end - 1 (the rate
// that just left that window; tn the time of the row just appended).
template <typename TF>
__device__ __forceinline__ void tail_update(const StepArgs<TF>& a, int v, int r, int64_t tn) {
  double* E = a.tail_acc + v * a.tail_len;
  for (int e = a.tail_src_ptr[r]; e < a.tail_src_ptr[r + 1]; ++e) {
    const int acc = a.tail_src[2 * e], Tend = a.tail_src[2 * e + 1];
    const int64_t t = tn - Tend - 1;
    if (t >= a.first) E[acc] += a.dt * a.ring64[(ring_slot(t, a.R) * a.nv + v) * a.N + r];
  }
}

// Long steps (gamma > 1 grid steps from n = time_new - gamma). Invariant between
// steps: an accumulator with upper lag T_end holds dt times the rows t <= n - T_end
// - 1. At the step's start (tail_advance) it takes the rows up to the step's
// evaluation head minus T_end + 1: the committed ones n - T_end .. n (from the
// ring) and the interior ones n+1 .. n+gamma-T_end-2 at the starting rate V^n; the
// commit (tail_commit_long) replaces those interior values by the averaged rate
// they are committed with and adds the row n+gamma-T_end-1, restoring the invariant.
template <typename TF>
__device__ __forceinline__ void tail_advance(const StepArgs<TF>& a, int v, int r, double Vn) {
  double* E = a.tail_acc + v * a.tail_len;
  const int64_t g = a.gamma, n = a.time_new - g;
  for (int e = a.tail_src_ptr[r]; e < a.tail_src_ptr[r + 1]; ++e) {
    const int acc = a.tail_src[2 * e], Tend = a.tail_src[2 * e + 1];
    const int64_t hi = n + g - Tend - 2 < n ? n + g - Tend - 2 : n;
    double add = 0.0;
    for (int64_t t = n - Tend > a.first ? n - Tend : a.first; t <= hi; ++t)
      add += a.dt * a.ring64[(ring_slot(t, a.R) * a.nv + v) * a.N + r];
    const int64_t c = g - Tend - 2 > 0 ? g - Tend - 2 : 0;
    E[acc] += add + (double)c * a.dt * Vn;
  }
}

template <typename TF>
__device__ __forceinline__ void tail_commit_long(const StepArgs<TF>& a, int v, int r, double Vn, double Vb) {
  double* E = a.tail_acc + v * a.tail_len;
  const int64_t g = a.gamma, n = a.time_new - g;
  for (int e = a.tail_src_ptr[r]; e < a.tail_src_ptr[r + 1]; ++e) {
    const int acc = a.tail_src[2 * e], Tend = a.tail_src[2 * e + 1];
    const int64_t c = g - Tend - 2 > 0 ? g - Tend - 2 : 0;
    const int64_t ts = n + g - Tend - 1;
    double add = (double)c * a.dt * (Vb - Vn);
    if (ts >= a.first) add += a.dt * (ts <= n ? a.ring64[(ring_slot(ts, a.R) * a.nv + v) * a.N + r] : Vb);
    E[acc] += add;
  }
}

// operand copy of a rate value
template <typename TF>
__device__ __forceinline__ TF to_op(double x) {
  return (TF)x;
}
template <>
__device__ __forceinline__ __bf16 to_op<__bf16>(double x) {
  return (__bf16)(float)x;
}

// One wave per (variant, element): inverse transform by the whole wave, then
// lane 0 solves.
template <typename TF>
__global__ void k_stage(StepArgs<TF> a, int stage) {
  const int lane = threadIdx.x & 63;
  const int rg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (rg >= a.N * a.nv) return;
  const int v = rg / a.N, r = rg - v * a.N;
  const int64_t o = (int64_t)v * a.N, e = o + r;
  const int k = a.fault_of[r];
  const SelfFaultDev f = a.sf[k];
  const int j = r - f.off;
  const double fself = idft_wave(f, a.F + (int64_t)v * a.n_modes + f.mode_off, a.tw + f.tw, j, lane);
  if (lane != 0) return;
  const double t_next = a.clk ? (double)(a.time_new + *a.clk) * a.dt : a.t_next;
  const double tau0 = a.tau0[e] + a.tau0_rate[e] * (t_next - (double)a.step0[v] * a.dt);
  const Friction& fr = a.fric;
  if (stage == 0) {  // predictor: delta*, theta* from the current rates
    const double V = a.V[e];
    const double th_s = a.exact_state ? state_after(a.theta[e], V, fr.Dc[e], a.dts, fr.eps[e])
                                      : a.theta[e] + a.dts * a.thdot[e];
    const double fint = a.f_hist[e] - a.eta * lag0_apply(a.l0_ptr, a.l0_col, a.l0_val, a.V + o, r);
    const double Vs = newton_lnV(tau0 + fself + fint, th_s, a.eta, fr.a[e], fr.b[e], fr.Dc[e], fr.sn[e], fr.V0[e],
                                 fr.f0[e], log(V), a.fail + v);
    const double tds = state_rate(Vs, th_s, fr.Dc[e], fr.eps[e]);
    a.Vstar[e] = Vs;
    a.Vbar[e] = 0.5 * (V + Vs);
    a.th2[e] = a.exact_state ? state_after(a.theta[e], 0.5 * (V + Vs), fr.Dc[e], a.dts, fr.eps[e])
                             : a.theta[e] + a.dts * 0.5 * (a.thdot[e] + tds);
  } else {  // corrector with the averaged rates; only the lag-0 terms change
    const double Vb = a.Vbar[e];
    const double th2 = a.th2[e];
    const double fint = a.f_hist[e] - a.eta * lag0_apply(a.l0_ptr, a.l0_col, a.l0_val, a.Vbar + o, r);
    const double V2 = newton_lnV(tau0 + fself + fint, th2, a.eta, fr.a[e], fr.b[e], fr.Dc[e], fr.sn[e], fr.V0[e],
                                 fr.f0[e], log(a.Vstar[e]), a.fail + v);
    (void)Vb;
    // the commit (k_commit) takes these once every solve of the variant is known to
    // have converged
    a.V2[e] = V2;
    a.td2[e] = state_rate(V2, th2, fr.Dc[e], fr.eps[e]);
    a.fs2[e] = fself;
    a.fi2[e] = fint;
  }
}

// Commit of the corrector, after every Newton solve of the step: threads
// [0, nv N) take one element each, the next nv n_modes one slip coefficient each.
// A variant whose flag is set (a solve of this or an earlier step failed) is left
// as it is: its state, histories and accumulators stay at its last good step.
template <typename TF>
__global__ void k_commit(StepArgs<TF> a) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = (int64_t)a.N * a.nv;
  const int64_t c = a.clk ? *a.clk : 0;
  if (g < ne) {
    const int v = (int)(g / a.N), r = (int)(g - (int64_t)v * a.N);
    if (a.fail[v]) return;
    const int64_t e = g;
    const double V2 = a.V2[e];
    if (a.tail && a.gamma > 1) tail_commit_long(a, v, r, a.V[e], a.Vbar[e]);
    a.delta[e] += a.dts * a.Vbar[e];
    a.theta[e] = a.th2[e];
    a.thdot[e] = a.td2[e];
    a.V[e] = V2;
    a.f_self_out[e] = a.fs2[e];
    a.f_int_out[e] = a.fi2[e];
    const int64_t tn = a.time_new + c;
    const int64_t sl = ring_slot(tn, a.R), ri = (sl * a.nv + v) * a.N + r;
    a.ring64[ri] = V2;
    if ((void*)a.ringop != (void*)a.ring64)
      a.ringop[a.op_vfast ? (sl * a.N + r) * a.nv + v : ri] = to_op<TF>(V2);
    if (a.tail && a.gamma == 1) tail_update(a, v, r, tn);
    if (r == 0) a.good[v] = tn;
    return;
  }
  g -= ne;
  if (g >= (int64_t)a.n_modes * a.nv) return;
  const int v = (int)(g / a.n_modes), gm = (int)(g - (int64_t)v * a.n_modes);
  if (a.fail[v]) return;
  const SelfMode md = a.modes[gm];
  if (md.W > 0) a.dring[v * a.dring_len + md.ring + ring_slot(a.self_head + c, md.W)] = a.Dnew[g];
}

// Prescribed mode, before the evaluation of step n: append V^{n-1}, advance slip.
// One thread per (variant, element).
template <typename TF>
__global__ void k_pre_push(StepArgs<TF> a, const double* __restrict__ Vin) {
  const int rg = blockIdx.x * blockDim.x + threadIdx.x;
  if (rg >= a.N * a.nv) return;
  const int v = rg / a.N, r = rg - v * a.N;
  const double x = Vin[rg];
  const int64_t sl = ring_slot(a.time_new, a.R), ri = (sl * a.nv + v) * a.N + r;
  a.ring64[ri] = x;
  if ((void*)a.ringop != (void*)a.ring64) a.ringop[a.op_vfast ? (sl * a.N + r) * a.nv + v : ri] = to_op<TF>(x);
  a.delta[rg] += a.dt * x;
  if (a.tail) tail_update(a, v, r, a.time_new);
}

// Prescribed mode output: f^n = f_self + f_hist - mu/(2cs) K^0 V^{n-1} (one wave
// per (variant, element)).
template <typename TF>
__global__ void k_pre_out(StepArgs<TF> a, const double* __restrict__ Vprev, double* __restrict__ fout) {
  const int lane = threadIdx.x & 63;
  const int rg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (rg >= a.N * a.nv) return;
  const int v = rg / a.N, r = rg - v * a.N;
  const int64_t o = (int64_t)v * a.N;
  const int k = a.fault_of[r];
  const SelfFaultDev f = a.sf[k];
  const double fself = idft_wave(f, a.F + (int64_t)v * a.n_modes + f.mode_off, a.tw + f.tw, r - f.off, lane);
  if (lane == 0) fout[rg] = fself + a.f_hist[rg] - a.eta * lag0_apply(a.l0_ptr, a.l0_col, a.l0_val, Vprev + o, r);
}

// Zero variant v's rows of a [rows][nv][N] array (16-bit words; zero bits are
// 0.0 in every floating-point format used here).
__global__ void k_clear_variant(uint16_t* __restrict__ base, int64_t rows, int64_t pitch, int64_t width,
                                int64_t off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * width) return;
  const int64_t r = i / width, c = i - r * width;
  base[r * pitch + off + c] = 0;
}

// ------------------------------------------------------------------ launchers

void launch_clear_variant(void* base, int64_t rows, int nv, int v, int N, int elem_bytes, hipStream_t s) {
  const int64_t w = (int64_t)N * elem_bytes / 2;  // 16-bit words per variant row
  const int64_t n = rows * w;
  if (n == 0) return;
  hipLaunchKernelGGL(k_clear_variant, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint16_t*)base, rows,
                     w * nv, w, w * v);
}

template <typename TF, int S>
static void hmat_s(int n, const void* items, const int32_t* lagT, const int32_t* lagCol, const int32_t* lagColOff,
                   const void* arena, const void* ring, int64_t head, int64_t R, int N, const double* tail_acc,
                   double* partials, int pstride, hipStream_t s, const int64_t* clk) {
  hipLaunchKernelGGL((k_hmat<TF, TF, S>), dim3(n), dim3(kItemThreads), 0, s, (const Item*)items, lagT, lagCol,
                     lagColOff, (const TF*)arena, (const TF*)ring, head, R, N, tail_acc, partials, pstride, clk);
}

template <typename TF>
static void hmat_t(int S, int n, const void* items, const int32_t* lagT, const int32_t* lagCol,
                   const int32_t* lagColOff, const void* arena, const void* ring, int64_t head, int64_t R, int N,
                   const double* tail_acc, double* partials, int ps, hipStream_t s, const int64_t* clk) {
  switch (S) {
    case 1: hmat_s<TF, 1>(n, items, lagT, lagCol, lagColOff, arena, ring, head, R, N, tail_acc, partials, ps, s, clk); break;
    case 2: hmat_s<TF, 2>(n, items, lagT, lagCol, lagColOff, arena, ring, head, R, N, tail_acc, partials, ps, s, clk); break;
    case 4: hmat_s<TF, 4>(n, items, lagT, lagCol, lagColOff, arena, ring, head, R, N, tail_acc, partials, ps, s, clk); break;
    case 8: hmat_s<TF, 8>(n, items, lagT, lagCol, lagColOff, arena, ring, head, R, N, tail_acc, partials, ps, s, clk); break;
    case 16: hmat_s<TF, 16>(n, items, lagT, lagCol, lagColOff, arena, ring, head, R, N, tail_acc, partials, ps, s, clk); break;
    default: break;
  }
}

void launch_hmat(const HostOp& h, int S, int n_items, const void* items, const int32_t* lagT, const int32_t* lagCol,
                 const int32_t* lagColOff, const void* arena, const void* ring, int64_t head,
                 const double* tail_acc, double* partials, int pstride, hipStream_t s, const int64_t* clk) {
  if (n_items == 0) return;
  if (h.prm.factor_dtype == SEAS_F32 && S == 16 && h.use_mfma) {
    hipLaunchKernelGGL(k_hmat_mfma16, dim3(n_items), dim3(kItemThreads), 0, s, (const Item*)items, lagT, lagCol,
                       lagColOff, (const float*)arena, (const float*)ring, head, (int64_t)h.ring_len, h.N,
                       (float*)partials, pstride, clk);
    return;
  }
  if (h.prm.factor_dtype == SEAS_F64)
    hmat_t<double>(S, n_items, items, lagT, lagCol, lagColOff, arena, ring, head, h.ring_len, h.N, tail_acc,
                   partials, pstride, s, clk);
  else
    hmat_t<float>(S, n_items, items, lagT, lagCol, lagColOff, arena, ring, head, h.ring_len, h.N, tail_acc,
                  partials, pstride, s, clk);
}

void launch_hmat_f32far(const HostOp& h, int n_items, const void* items, const int32_t* lagT, const int32_t* lagCol,
                        const int32_t* lagColOff, const float* arena, const void* ring, int64_t head,
                        float* partials, hipStream_t s, const int64_t* clk) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_hmat_mfma16, dim3(n_items), dim3(kItemThreads), 0, s, (const Item*)items, lagT, lagCol,
                     lagColOff, arena, (const float*)ring, head, (int64_t)h.ring_len, h.N, partials, 16, clk);
}

bool far_partials_f32(const HostOp& h, int S) {
  return h.seg || (h.prm.factor_dtype == SEAS_F32 && S == 16 && h.use_mfma);
}


template <typename TP>
static void reduce_far_t(const HostOp& h, int S, const TP* partials, const int32_t* ptr, const int32_t* idx, double* f,
                         hipStream_t s) {
  const dim3 g(blocks_for(h.N, 4)), b(256);
  switch (S) {
    case 1: hipLaunchKernelGGL((k_reduce_far<1, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 2: hipLaunchKernelGGL((k_reduce_far<2, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 4: hipLaunchKernelGGL((k_reduce_far<4, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 8: hipLaunchKernelGGL((k_reduce_far<8, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 16: hipLaunchKernelGGL((k_reduce_far<16, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 32: hipLaunchKernelGGL((k_reduce_far<32, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    case 64: hipLaunchKernelGGL((k_reduce_far<64, TP>), g, b, 0, s, partials, ptr, idx, h.N, -h.eta, f); break;
    default: break;
  }
}

void launch_reduce_far(const HostOp& h, int S, const void* partials, bool f32, const int32_t* ptr,
                       const int32_t* idx, double* f, hipStream_t s) {
  if (f32) reduce_far_t(h, S, (const float*)partials, ptr, idx, f, s);
  else reduce_far_t(h, S, (const double*)partials, ptr, idx, f, s);
}

void launch_reduce_near(const HostOp& h, const double* partials, const int32_t* ptr, const int32_t* idx,
                        const double* base, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_near, dim3(blocks_for(h.N, 4)), dim3(256), 0, s, partials, ptr, idx, h.N, -h.eta, base,
                     f);
}

void launch_self_hist(int n_modes, int nv, int64_t dring_len, const SelfMode* modes, const double* tab,
                      const double2* dring, int64_t time0, double2* Fh, hipStream_t s, const int64_t* clk) {
  hipLaunchKernelGGL(k_self_hist, dim3(blocks_for((int64_t)n_modes * nv, 4)), dim3(256), 0, s, modes, n_modes, nv,
                     dring_len, tab, dring, time0, Fh, clk);
}

void launch_dft(int n_modes, int nv, int N, int64_t dring_len, const SelfMode* modes, const SelfFaultDev* sf,
                const double* delta, const double* vel, double coef, const double2* tw, const double* tab,
                const double2* Fh, double2* Fout, double2* dring, int push, int64_t push_time, int64_t ring_head,
                hipStream_t s, double2* Dsave, const int64_t* clk) {
  hipLaunchKernelGGL(k_dft, dim3(blocks_for((int64_t)n_modes * nv, 4)), dim3(256), 0, s, modes, n_modes, nv, N,
                     dring_len, sf, delta, vel, coef, tw, tab, Fh, Fout, dring, push, push_time, ring_head, Dsave,
                     clk);
}

__global__ void k_clock(int64_t* __restrict__ clk, int64_t v, int add) {
  if (threadIdx.x == 0) *clk = add ? *clk + v : v;
}

void launch_clock(int64_t* clk, int64_t v, int add, hipStream_t s) {
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, s, clk, v, add);
}

__global__ void k_dt_ev(const double* __restrict__ V, const double* __restrict__ Dc, int64_t ne, double xi,
                        double* __restrict__ part) {
  __shared__ double wmin[4];
  double m = INFINITY;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x)
    m = fmin(m, xi * Dc[e] / V[e]);
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
}

template <typename TF>
__global__ void k_tail_advance(StepArgs<TF> a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)a.N * a.nv) return;
  const int v = (int)(g / a.N), r = (int)(g - (int64_t)v * a.N);
  if (a.fail[v]) return;
  tail_advance(a, v, r, a.V[g]);
}

template <typename TF>
__global__ void k_fill_rows(StepArgs<TF> a, int64_t lo, int64_t rows, const double* __restrict__ src) {
  const int64_t ne = (int64_t)a.N * a.nv;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= rows * ne) return;
  const int64_t k = g / ne, e = g - k * ne;
  const int v = (int)(e / a.N), r = (int)(e - (int64_t)v * a.N);
  const double x = src[e];
  const int64_t sl = ring_slot(lo + k, a.R), ri = (sl * a.nv + v) * a.N + r;
  a.ring64[ri] = x;
  if ((void*)a.ringop != (void*)a.ring64) a.ringop[a.op_vfast ? (sl * a.N + r) * a.nv + v : ri] = to_op<TF>(x);
}

__global__ void k_fill_modes(int n_modes, int nv, int64_t dring_len, const SelfMode* __restrict__ modes,
                             double2* __restrict__ dring, int64_t n, int64_t gamma, const double2* __restrict__ Dend,
                             double2* __restrict__ Dsv, int commit) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n_modes * nv) return;
  const int v = (int)(g / n_modes), gm = (int)(g - (int64_t)v * n_modes);
  const SelfMode md = modes[gm];
  if (md.W <= 0) return;
  double2* ring = dring + v * dring_len + md.ring;
  double2 d0;
  if (commit) {
    d0 = Dsv[g];
  } else {
    d0 = ring[ring_slot(n, md.W)];
    Dsv[g] = d0;
  }
  const double2 d1 = Dend[g];
  // the entries the next history sums read: predictor n+gamma-W .. n+gamma-1, after
  // the commit n+gamma-W+1 .. n+gamma-1 (its push adds n+gamma); interior only
  const int64_t m0 = commit ? gamma - md.W + 1 : gamma - md.W;
  for (int64_t m = m0 > 1 ? m0 : 1; m < gamma; ++m) {
    const double w = (double)m / (double)gamma;
    ring[ring_slot(n + m, md.W)] = make_double2(d0.x + w * (d1.x - d0.x), d0.y + w * (d1.y - d0.y));
  }
}

void launch_dt_ev(const double* V, const double* Dc, int64_t ne, double xi, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_ev, dim3(nblocks), dim3(256), 0, s, V, Dc, ne, xi, part);
}

template <typename TF>
void launch_tail_advance(const StepArgs<TF>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_tail_advance<TF>), dim3(blocks_for((int64_t)a.N * a.nv, 256)), dim3(256), 0, s, a);
}

template <typename TF>
void launch_fill_rows(const StepArgs<TF>& a, int64_t lo, int64_t hi, const double* src, hipStream_t s) {
  if (hi < lo) return;
  const int64_t rows = hi - lo + 1;
  hipLaunchKernelGGL((k_fill_rows<TF>), dim3(blocks_for(rows * a.N * a.nv, 256)), dim3(256), 0, s, a, lo, rows,
                     src);
}

void launch_fill_modes(int n_modes, int nv, int64_t dring_len, const SelfMode* modes, double2* dring, int64_t n,
                       int64_t gamma, const double2* Dend, double2* Dsv, int commit, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_modes, dim3(blocks_for((int64_t)n_modes * nv, 256)), dim3(256), 0, s, n_modes, nv,
                     dring_len, modes, dring, n, gamma, Dend, Dsv, commit);
}

template <typename TF>
void launch_stage(const StepArgs<TF>& a, int stage, hipStream_t s) {
  hipLaunchKernelGGL((k_stage<TF>), dim3(blocks_for((int64_t)a.N * a.nv, 4)), dim3(256), 0, s, a, stage);
}

template <typename TF>
void launch_commit(const StepArgs<TF>& a, hipStream_t s) {
  const int64_t n = (int64_t)a.N * a.nv + (int64_t)a.n_modes * a.nv;
  hipLaunchKernelGGL((k_commit<TF>), dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
}

template <typename TF>
void launch_prescribed_push(const StepArgs<TF>& a, const double* Vin, hipStream_t s) {
  hipLaunchKernelGGL((k_pre_push<TF>), dim3(blocks_for((int64_t)a.N * a.nv, 256)), dim3(256), 0, s, a, Vin);
}

template <typename TF>
void launch_prescribed_out(const StepArgs<TF>& a, const double* Vprev, double* fout, hipStream_t s) {
  hipLaunchKernelGGL((k_pre_out<TF>), dim3(blocks_for((int64_t)a.N * a.nv, 4)), dim3(256), 0, s, a, Vprev, fout);
}

template void launch_tail_advance<double>(const StepArgs<double>&, hipStream_t);
template void launch_tail_advance<float>(const StepArgs<float>&, hipStream_t);
template void launch_tail_advance<__bf16>(const StepArgs<__bf16>&, hipStream_t);
template void launch_fill_rows<double>(const StepArgs<double>&, int64_t, int64_t, const double*, hipStream_t);
template void launch_fill_rows<float>(const StepArgs<float>&, int64_t, int64_t, const double*, hipStream_t);
template void launch_fill_rows<__bf16>(const StepArgs<__bf16>&, int64_t, int64_t, const double*, hipStream_t);
template void launch_commit<double>(const StepArgs<double>&, hipStream_t);
template void launch_commit<float>(const StepArgs<float>&, hipStream_t);
template void launch_commit<__bf16>(const StepArgs<__bf16>&, hipStream_t);
template void launch_stage<double>(const StepArgs<double>&, int, hipStream_t);
template void launch_stage<float>(const StepArgs<float>&, int, hipStream_t);
template void launch_stage<__bf16>(const StepArgs<__bf16>&, int, hipStream_t);
template void launch_prescribed_push<double>(const StepArgs<double>&, const double*, hipStream_t);
template void launch_prescribed_push<float>(const StepArgs<float>&, const double*, hipStream_t);
template void launch_prescribed_push<__bf16>(const StepArgs<__bf16>&, const double*, hipStream_t);
template void launch_prescribed_out<double>(const StepArgs<double>&, const double*, double*, hipStream_t);
template void launch_prescribed_out<float>(const StepArgs<float>&, const double*, double*, hipStream_t);
template void launch_prescribed_out<__bf16>(const StepArgs<__bf16>&, const double*, double*, hipStream_t);

}  // namespace seas
