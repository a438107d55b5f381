// Segment far-list pass on the matrix cores (BF16 / FP16 factors, and FP32
// factors with 16 or 32 windows) and its launcher.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace seas {

// ------------------------------------------------------------------ segment matrix-core form
// BF16 / FP16 factors (one power-of-two scale per item) times a 16-bit copy of
// the history, v_mfma_f32_16x16x32_{bf16,f16}, FP32 accumulation; or FP32
// factors times the FP32 history, eight v_mfma_f32_16x16x4_f32 per step. The
// products have NC = 16 NT columns: S history windows of nv variants, column
// n = k nv + v. Operand layout of one step (16 rows x 32 inner x 16 columns):
//   A: lane l holds A[row l%16][8 (l/16) .. +7]      (one 16- or 32-byte load)
//   B: lane l holds B[8 (l/16) .. +7][column l%16]   (one 16- or 32-byte LDS read)
//   D: lane l, register v holds D[row 4 (l/16) + v][column l%16]
// (FP32: MFMA s of the step takes value s of each lane's eight, so lane group g
// feeds inner index 8 g + s to the instruction's inner slot g; every inner index
// of the step meets its own B value once.)
// Factors are stored with the inner index fastest and rows padded to multiples
// of 8 values, so both operands are aligned 16-byte vectors:
//   dense    [p][nlag * q8]   inner index e = l q8 + j (lag l, source j)
//   low rank W [ncol][q8], then U [p][ncol8]
// The staged history holds, for rows r (time tnew - r, newest first), variants v
// and sources j, the value at LDS index (r nv + v) ldh + j, where the row stride
// ldh is q8 padded to an odd number of 16-byte groups (the 16 rows an operand
// reads then fall in distinct banks); B(e, n) for lag l, window k, variant v is
// row l + S - 1 - k, i.e. index l nv ldh + j + hoff(n) with
// hoff(n) = ((S - 1 - k) nv + v) ldh.
// A workgroup runs a segment: consecutive items with the same receiver rows.
// Each wave keeps the sums of its row tiles in registers across the segment
// (rows up to 4 x RW tiles; larger blocks come as single-item segments whose row
// tiles are written as they finish) and one partial set of p x NC values is
// written per segment.
template <typename T16>
struct Mx;
template <>
struct Mx<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ mfma_f4 mma(v8 a, v8 b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ __bf16 cvt(float x) { return (__bf16)x; }
};
template <>
struct Mx<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ mfma_f4 mma(v8 a, v8 b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
};
template <>
struct Mx<float> {
  typedef float v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ mfma_f4 mma(v8 a, v8 b, mfma_f4 c) {
#pragma unroll
    for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
    return c;
  }
  static __device__ __forceinline__ float cvt(float x) { return x; }
};

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// power of two >= m (1 for m = 0)
__device__ __forceinline__ float pow2_at_least(float m) {
  if (!(m > 0.0f)) return 1.0f;
  int e;
  (void)frexpf(m, &e);
  return ldexpf(1.0f, e);
}

// tmp[t] += sum over inner k in [k0, k1) of A(k) B(k, t); k0, k1 multiples of 8.
// 16-bit values: the global operand of PF steps of 32 is loaded before their
// MFMAs (one round trip for most items). FP32 values: the global operand runs PF
// steps ahead in a rolling buffer, slot s refilled for the next batch as soon as
// its step's MFMAs are issued, so a wave keeps about PF steps of loads in flight
// throughout (the 16-bit instances have no registers to spare for it). The LDS
// operand is read step by step.
template <typename T16, int NT, int PF, typename FA, typename FB>
__device__ __forceinline__ void x16_kloop(int k0, int k1, FA A, FB B, mfma_f4 (&tmp)[NT], int g) {
  typedef typename Mx<T16>::v8 v8;
  const v8 zero = {};
  if constexpr (sizeof(T16) == 4) {
    v8 a[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      const int kk = k0 + 32 * s + 8 * g;
      a[s] = kk < k1 ? A(kk) : zero;
    }
    for (int k = k0; k < k1; k += 32 * PF) {
#pragma unroll
      for (int s = 0; s < PF; ++s) {
        if (k + 32 * s >= k1) break;  // the same for every lane of the wave
        const int kk = k + 32 * s + 8 * g;
        const bool ok = kk < k1;
#pragma unroll
        for (int t = 0; t < NT; ++t) tmp[t] = Mx<T16>::mma(a[s], ok ? B(kk, t) : zero, tmp[t]);
        const int kn = kk + 32 * PF;
        a[s] = kn < k1 ? A(kn) : zero;
      }
    }
  } else {
    for (int k = k0; k < k1; k += 32 * PF) {
      v8 a[PF];
#pragma unroll
      for (int s = 0; s < PF; ++s) {
        const int kk = k + 32 * s + 8 * g;
        a[s] = kk < k1 ? A(kk) : zero;
      }
#pragma unroll
      for (int s = 0; s < PF; ++s) {
        if (k + 32 * s >= k1) break;  // the same for every lane of the wave
        const int kk = k + 32 * s + 8 * g;
        const bool ok = kk < k1;
#pragma unroll
        for (int t = 0; t < NT; ++t) tmp[t] = Mx<T16>::mma(a[s], ok ? B(kk, t) : zero, tmp[t]);
      }
    }
  }
}

// Tuned variants of the operator's far kernel (seas_operator_tune): the prefetch
// depth of the global operand and, for the FP32 one-variant instances, the waves
// per SIMD the registers are fitted to. The arithmetic and its order are the same
// in every variant.
//   FP32:   0: prefetch 2 steps, 4 waves (the 32-window instance spills 12 VGPRs
//              for it); 1: prefetch 2 steps, 3 waves; 2: prefetch 3 steps, 3 waves
//   16-bit: 0: prefetch 8 steps; 1: 4 steps; 2: 12 steps (waves as untuned)
constexpr int x16_pf(int eb, int tune) { return eb == 4 ? (tune == 2 ? 3 : 2) : (tune == 1 ? 4 : tune == 2 ? 12 : 8); }
constexpr int x16_waves(bool scale, int nt, bool vfast, bool win, int tune) {
  return (nt == 1 && !vfast) ? (scale ? 3 : (tune == 0 ? 4 : 3)) : (win ? (tune == 0 ? 4 : 3) : 2);
}

// WIN: one variant's time windows (NT = 2: 32 windows of FP32 factors), staged
// with the 16-column budget so that four workgroups share a CU
template <typename T16, typename TR, bool SCALE, int NT, bool VFAST, bool WIN, int TUNE>
__global__ __launch_bounds__(kItemThreads) __attribute__((amdgpu_waves_per_eu(x16_waves(SCALE, NT, VFAST, WIN, TUNE)))) void k_hmat_x16(
    const Item* __restrict__ items, const int32_t* __restrict__ seg_ptr, const int32_t* __restrict__ lagT,
    const int32_t* __restrict__ lagCol, const int32_t* __restrict__ lagColOff, const T16* __restrict__ arena,
    const TR* __restrict__ ring, int64_t head, int64_t R, int N, int S, int nv,
    const double* __restrict__ tail_acc, int64_t tail_len, float* __restrict__ partials,
    const int64_t* __restrict__ clk) {
  if (clk) head += *clk;
  typedef typename Mx<T16>::v8 v8;
  constexpr int NC = 16 * NT;
  constexpr int EB = (int)sizeof(T16);  // bytes per stored value
  constexpr int G = 16 / EB;            // values per 16-byte group
  constexpr int RW = NT == 1 ? 8 : 4;   // row tiles per wave held across a segment
  constexpr int PF = x16_pf(EB, TUNE);  // inner steps whose global operand is loaded ahead
  // staged history and projected values (seg_hist_limit, seg_z_limit + 16 bytes):
  // the same bytes for every value type
  constexpr int HL = (NT >= 2 && !WIN ? 2 * kHist16 : kHist16) * 2 / EB;
  __shared__ __attribute__((aligned(16))) T16 h[HL];
  constexpr int ZL = (NT >= 2 && !WIN ? 2 * kZ16 : kZ16) * 2 / EB;
  __shared__ __attribute__((aligned(16))) T16 z[ZL];
  // the staging maxima live at the end of z, which projected panels never use:
  // one per wave (smax), or one per variant (smv) for scaled ensemble panels
  float* smax = reinterpret_cast<float*>(z + ZL - G);
  float* smv = reinterpret_cast<float*>(z + ZL) - nv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, g = lane >> 4;
  const int nv_shift = __builtin_ctz((unsigned)nv);  // nv is a power of two
  const int x0 = seg_ptr[blockIdx.x], x1 = seg_ptr[blockIdx.x + 1];
  const int p = items[x0].p;
  const int RT = (p + 15) >> 4;
  // Work units: (row tile, inner-range split) pairs, KS splits per tile, unit
  // id = tile * KS + split; wave w takes units w, w + 4, ... KS is the smallest
  // of 1, 2, 4 that makes the unit count a multiple of 4 (all waves equally
  // busy), as long as each wave holds at most RW units and the split sums fit
  // the LDS reduction buffer; tall blocks keep KS = 1.
  int KS = 1;
  if ((RT & 3) != 0) {
    const int k = (RT & 1) ? 4 : 2;
    if ((RT * k + 3) / 4 <= RW && RT * k * NT <= 32) KS = k;
  }
  const int units = RT * KS;
  const int my_units = (units - wave + 3) / 4;
  const bool held = my_units <= RW;          // else a single-item segment (KS = 1), written per unit
  float* out = partials + items[x0].part;
  mfma_f4 acc[RW][NT];
#pragma unroll
  for (int u = 0; u < RW; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[u][t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};

  for (int x = x0; x < x1; ++x) {
    const Item it = items[x];
    const int q = it.q, q8 = (q + 7) & ~7, nl = it.nlag;
    const int ldh = ((q8 / G) & 1) ? q8 : q8 + G;  // LDS row stride (seg_ld)
    const int span = it.src == 0 ? nl + S - 1 : 1;
    const int nrow = span * nv;
    const int64_t tnew = head + S - 1 - lagT[it.lag_off];
    __syncthreads();  // the previous item is done with h and z
    // ---- stage the history panel (16-bit, scaled by 1/hs for FP16). Flat over
    // the nrow x q8 panel: value e is row rv = e / q8 (time tnew - rv / nv,
    // variant rv % nv), source j = e % q8; each thread issues 8 loads before it
    // uses them, so a workgroup keeps 2048 loads in flight.
    const int tot = nrow * q8;
    const float inv_q8s = 1.0f / (float)q8;
    const int64_t s0 = ring_slot(tnew, R);
    auto hval = [&](int e) -> float {
      const int rv = (int)(((float)e + 0.5f) * inv_q8s), j = e - rv * q8;
      if (j >= q) return 0.0f;
      if (it.src != 0) return (float)tail_acc[(int64_t)rv * tail_len + it.tail_off + j];
      const int r = rv >> nv_shift, v = rv - (r << nv_shift);
      int64_t sl = s0 - r;
      if (sl < 0) sl += R;  // r < R
      return (float)ring[(sl * nv + v) * (int64_t)N + it.col0 + j];
    };
    float hs = 1.0f;
    // scaled ensembles (S = 1): every staged row belongs to one variant, so each
    // variant's rows get their own power of two, and a variant slipping fast does
    // not push another's small rates below FP16's range
    const bool per_variant = SCALE && nv > 1;
    if (per_variant) {
      for (int v = tid; v < nv; v += kItemThreads) smv[v] = 0.0f;
      __syncthreads();
      for (int e0 = tid; e0 < tot; e0 += 8 * kItemThreads) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kItemThreads;
          x[u] = e < tot ? hval(e) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kItemThreads;
          if (e < tot) {
            const int rv = (int)(((float)e + 0.5f) * inv_q8s);
            // non-negative floats order like their bit patterns
            atomicMax(reinterpret_cast<int*>(smv + (rv & (nv - 1))), __float_as_int(fabsf(x[u])));
          }
        }
      }
      __syncthreads();
      for (int v = tid; v < nv; v += kItemThreads) smv[v] = pow2_at_least(smv[v]);
      __syncthreads();
      for (int e0 = tid; e0 < tot; e0 += 8 * kItemThreads) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kItemThreads;
          x[u] = e < tot ? hval(e) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kItemThreads;
          if (e < tot) {
            const int rv = (int)(((float)e + 0.5f) * inv_q8s);
            h[e + rv * (ldh - q8)] = Mx<T16>::cvt(x[u] / smv[rv & (nv - 1)]);
          }
        }
      }
    } else if (VFAST && it.src == 0) {
      // 16-bit history copy laid out [R][N][nv]. A thread takes a tile of 8
      // sources x 8 variants: 8 aligned 16-byte loads (one per source, 8 variants
      // each; the 8 lanes of a group read one 128-byte row segment), a transpose
      // in registers, and 8 aligned 16-byte LDS stores (one per variant, 8
      // consecutive sources). Tiles u = ((r nj + jg) ng + vg), nj = q8 / 8.
      typedef uint16_t u8v __attribute__((ext_vector_type(8)));
      const int ng = nv >> 3, nj = q8 >> 3, nt = span * nj * ng;
      const float inv_nj = 1.0f / (float)nj;
      for (int u = tid; u < nt; u += kItemThreads) {
        const int vg = u & (ng - 1), rest = u >> (nv_shift - 3);
        const int r = (int)(((float)rest + 0.5f) * inv_nj), jg = rest - r * nj;
        int64_t sl = s0 - r;
        if (sl < 0) sl += R;
        const uint16_t* src = (const uint16_t*)ring + ((sl * N + it.col0 + 8 * jg) * nv + vg * 8);
        u8v xv[8], yv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) xv[k] = (8 * jg + k < q) ? *(const u8v*)(src + (int64_t)k * nv) : u8v{};
#pragma unroll
        for (int v = 0; v < 8; ++v)
#pragma unroll
          for (int k = 0; k < 8; ++k) yv[v][k] = xv[k][v];
        uint16_t* d = (uint16_t*)h + ((r * nv + vg * 8) * ldh + 8 * jg);
#pragma unroll
        for (int v = 0; v < 8; ++v) *(u8v*)(d + v * ldh) = yv[v];
      }
    } else if (SCALE && tot <= 16 * kItemThreads) {
      // FP16, panels of up to 16 values per thread: one pass, values kept in
      // registers while the panel's maximum is formed
      float xs[16];
      float m = 0.0f;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + u * kItemThreads;
        xs[u] = e < tot ? hval(e) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) m = fmaxf(m, fabsf(xs[u]));
      m = wave_max(m);
      if (lane == 0) smax[wave] = m;
      __syncthreads();
      hs = pow2_at_least(fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3])));
      const float hsi = 1.0f / hs;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + u * kItemThreads;
        if (e < tot) {
          const int rv = (int)(((float)e + 0.5f) * inv_q8s);
          h[e + rv * (ldh - q8)] = Mx<T16>::cvt(xs[u] * hsi);
        }
      }
    } else {
    if (SCALE) {
      float m = 0.0f;
      for (int e0 = tid; e0 < tot; e0 += 8 * kItemThreads) {
        float x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * kItemThreads;
          x[u] = e < tot ? hval(e) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) m = fmaxf(m, fabsf(x[u]));
      }
      m = wave_max(m);
      if (lane == 0) smax[wave] = m;
      __syncthreads();
      hs = pow2_at_least(fmaxf(fmaxf(smax[0], smax[1]), fmaxf(smax[2], smax[3])));
    }
    const float hsi = 1.0f / hs;
    for (int e0 = tid; e0 < tot; e0 += 8 * kItemThreads) {
      float x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kItemThreads;
        x[u] = e < tot ? hval(e) : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * kItemThreads;
        if (e < tot) {
          const int rv = (int)(((float)e + 0.5f) * inv_q8s);
          h[e + rv * (ldh - q8)] = Mx<T16>::cvt(x[u] * hsi);
        }
      }
    }
    }
    // column offsets of this lane's N-tiles
    int hoff[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + l16, k = n / nv, v = n - k * nv;
      hoff[t] = ((S - 1 - k) * nv + v) * ldh;
    }
    __syncthreads();
    const T16* base = arena + it.data;
    float sc = it.scale * hs;
    // the scale of each of this lane's product columns (column n = variant n when
    // per_variant)
    float sct[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) sct[t] = per_variant ? it.scale * smv[(t * 16 + l16) & (nv - 1)] : sc;
    int E, stride, zld = 0;
    const T16* M;
    if (it.kind == 0) {
      // ---- projection Z_l = W_l H_l per lag, column tiles of 16 round robin over waves
      const int nc = it.ncol, nc8 = (nc + 7) & ~7;
      const int ldz = ((nc8 / G) & 1) ? nc8 : nc8 + G;  // LDS row stride of Z (seg_ld)
      const int32_t* cp = lagCol + lagColOff[x];
      float zs = 1.0f;
      if (SCALE) {
        zs = 1.0f / pow2_at_least((float)q8);
        sc /= zs;
#pragma unroll
        for (int t = 0; t < NT; ++t) sct[t] /= zs;
      }
      // Lag l has ceil(rank_l / 16) tiles of 16 columns; the item's tiles, numbered
      // lag after lag, are dealt round robin to the waves. A wave runs its tiles as
      // one stream of fragments (tile, step of 32 inner indices) with the global
      // operand of PB fragments loaded per round trip, so short tiles (one or two
      // steps) share their load latency. The lag of a tile comes from a prefix of
      // the tile counts of up to 63 lags held one per lane.
      constexpr int PB = EB == 4 ? 4 : 6;
      const int nst = (q8 + 31) >> 5;  // fragments per tile
      mfma_f4 tmp[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) tmp[t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
      int tiles_before = 0;
      for (int lc0 = 0; lc0 < nl; lc0 += 63) {
        const int nlc = min(63, nl - lc0);
        const int cpa = lane <= nlc ? cp[lc0 + lane] : 0;  // first column of lag lc0 + lane
        const int cpb = __shfl_down(cpa, 1, 64);            // its end (lanes < nlc)
        const int nt = lane < nlc ? (cpb - cpa + 15) >> 4 : 0;
        int incl = nt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        const int excl = incl - nt;  // tiles of the chunk before lag lc0 + lane
        const int T = __shfl(incl, 63, 64);
        const int first = (wave - tiles_before) & 3;  // this wave's first tile of the chunk
        const int F = (T > first ? (T - first + 3) / 4 : 0) * nst;
        for (int f0 = 0; f0 < F; f0 += PB) {
          v8 a[PB];
          int dl[PB], dc0[PB], dce[PB];  // tile of each fragment: lag in the chunk, columns
          int tl = f0 / nst, st = f0 - tl * nst;
#pragma unroll
          for (int b = 0; b < PB; ++b) {
            const int tt = first + 4 * tl;
            const int lr = __popcll(__ballot(lane < nlc && excl <= tt)) - 1;
            dl[b] = lr;
            dc0[b] = __builtin_amdgcn_readlane(cpa, lr) + 16 * (tt - __builtin_amdgcn_readlane(excl, lr));
            dce[b] = __builtin_amdgcn_readlane(cpb, lr);
            const int c = dc0[b] + l16, kk = 32 * st + 8 * g;
            a[b] = (f0 + b < F && c < dce[b] && kk < q8) ? *(const v8*)(base + (int64_t)c * q8 + kk) : v8{};
            if (++st == nst) {
              st = 0;
              ++tl;
            }
          }
          st = f0 - (f0 / nst) * nst;
#pragma unroll
          for (int b = 0; b < PB; ++b) {
            if (f0 + b >= F) break;  // the same for every lane of the wave
            if (st == 0) {
#pragma unroll
              for (int t = 0; t < NT; ++t) tmp[t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
            }
            const int kk = 32 * st + 8 * g;
            const bool ok = kk < q8;
            const int lofs = (lc0 + dl[b]) * nv * ldh;
#pragma unroll
            for (int t = 0; t < NT; ++t)
              tmp[t] = Mx<T16>::mma(a[b], ok ? *(const v8*)(h + lofs + kk + hoff[t]) : v8{}, tmp[t]);
            if (st == nst - 1) {
#pragma unroll
              for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  const int cc = dc0[b] + 4 * g + v;
                  if (cc < dce[b]) z[(t * 16 + l16) * ldz + cc] = Mx<T16>::cvt(tmp[t][v] * zs);
                }
              }
            }
            if (++st == nst) st = 0;
          }
        }
        tiles_before += T;
      }
      for (int e = tid; e < NC * (nc8 - nc); e += kItemThreads) {  // zero pad columns
        const int n = e / (nc8 - nc), c = nc + e - n * (nc8 - nc);
        z[n * ldz + c] = Mx<T16>::cvt(0.0f);
      }
      __syncthreads();
      M = base + (int64_t)nc * q8;
      E = nc8;
      stride = nc8;
      zld = ldz;
    } else {
      M = base;
      E = nl * q8;
      stride = nl * q8;
    }
    // ---- expansion / dense product: Y (p x NC) += sc * M (p x E) B (E x NC)
    const float inv_q8 = 1.0f / (float)q8;
    const int lag_stride = nv * ldh - q8;  // h index of (lag l, source j): l nv ldh + j = kk + l lag_stride
    for (int u = 0; u < my_units; ++u) {
      const int id = wave + 4 * u, rt = id / KS, ks = id - rt * KS;
      int k0 = ((int)((int64_t)(E / 8) * ks / KS)) * 8;
      int k1 = ((int)((int64_t)(E / 8) * (ks + 1) / KS)) * 8;
      if (it.kind == 0 && KS > 1) {
        // low rank: the inner range (ncol8) is short, so a row tile is not split;
        // its whole range goes to one of its KS units, chosen so that tiles
        // rt = 0, 1, 2, 3 land on waves 0, 2, 1, 3 (KS = 2) or 0, 1, 2, 3 (KS = 4)
        const int pick = KS == 4 ? (rt & 3) : ((rt & 3) >> 1);
        if (ks != pick) continue;  // the same for every lane of the wave
        k0 = 0;
        k1 = E;
      }
      const int i = rt * 16 + l16;
      const T16* arow = M + (int64_t)min(i, p - 1) * stride;
      mfma_f4 tmp[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) tmp[t] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
      auto A = [&](int kk) { return i < p ? *(const v8*)(arow + kk) : v8{}; };
      if (it.kind == 0) {
        x16_kloop<T16, NT, PF>(k0, k1, A, [&](int kk, int t) { return *(const v8*)(z + (t * 16 + l16) * zld + kk); },
                               tmp, g);
      } else if (nv == 1 && ldh == q8) {
        x16_kloop<T16, NT, PF>(k0, k1, A, [&](int kk, int t) { return *(const v8*)(h + kk + hoff[t]); }, tmp, g);
      } else {
        x16_kloop<T16, NT, PF>(
            k0, k1, A,
            [&](int kk, int t) {
              const int l = (int)(((float)kk + 0.5f) * inv_q8);
              return *(const v8*)(h + kk + l * lag_stride + hoff[t]);
            },
            tmp, g);
      }
      if (held) {
#pragma unroll
        for (int uu = 0; uu < RW; ++uu) {
          if (uu == u) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[uu][t] += sct[t] * tmp[t];
          }
        }
      } else {  // single-item segment of a tall block (wide): write this row tile
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ii = rt * 16 + 4 * g + v;
            if (ii < p) out[ii * NC + t * 16 + l16] = sct[t] * tmp[t][v];
          }
        }
      }
    }
  }
  if (!held) return;  // single-item segment of a tall block: written per unit above
  if (KS == 1) {
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      if (u >= my_units) break;
      const int rt = wave + 4 * u;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = rt * 16 + 4 * g + v;
          if (ii < p) out[ii * NC + t * 16 + l16] = acc[u][t][v];
        }
      }
    }
    return;
  }
  // inner-range splits: add the KS sums of each tile in split order through LDS
  float* red = reinterpret_cast<float*>(h);  // units x NT x 256 floats <= 32 KB <= sizeof h
  __syncthreads();
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    if (u >= my_units) break;
    const int id = wave + 4 * u;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(id * NT + t) * 256 + lane * 4 + v] = acc[u][t][v];
    }
  }
  __syncthreads();
  for (int e = tid; e < RT * NT * 256; e += kItemThreads) {
    const int rt = e / (NT * 256), rem = e - rt * NT * 256, t = rem >> 8, w = rem & 255, ln = w >> 2, v = w & 3;
    float sum = 0.0f;
    for (int kk = 0; kk < KS; ++kk) sum += red[((rt * KS + kk) * NT + t) * 256 + ln * 4 + v];
    const int ii = rt * 16 + 4 * (ln >> 4) + v;
    if (ii < p) out[ii * NC + t * 16 + (ln & 15)] = sum;
  }
}

template <typename T16, typename TR, bool SCALE, int NT, bool VFAST = false, bool WIN = false, int TUNE = 0>
static void x16_launch(const HostOp& h, const void* items, const int32_t* seg_ptr, const int32_t* lagT,
                       const int32_t* lagCol, const int32_t* lagColOff, const void* arena, const void* ring,
                       int64_t head, const double* tail_acc, float* partials, hipStream_t s, int nseg,
                       const int64_t* clk) {
  hipLaunchKernelGGL((k_hmat_x16<T16, TR, SCALE, NT, VFAST, WIN, TUNE>), dim3(nseg), dim3(kItemThreads), 0, s, (const Item*)items,
                     seg_ptr, lagT, lagCol, lagColOff, (const T16*)arena, (const TR*)ring, head, (int64_t)h.ring_len,
                     h.N, h.time_block, h.n_variants, tail_acc, (int64_t)h.tail_len, partials, clk);
}

void launch_hmat_x16(const HostOp& h, const void* items, const int32_t* seg_ptr, int nseg, const int32_t* lagT,
                     const int32_t* lagCol, const int32_t* lagColOff, const void* arena, const void* ring,
                     int64_t head, const double* tail_acc, float* partials, hipStream_t s, const int64_t* clk) {
  if (nseg < 1) return;
  const bool bf = h.prm.factor_dtype == SEAS_BF16;
  if (!h.x16) {  // FP32 factors, one variant, 16 or 32 windows, in the operator's tuned variant
#define SEAS_X16_F32(TU)                                                                                      \
  if (h.ncols == 32)                                                                                          \
    x16_launch<float, float, false, 2, false, true, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, ring, \
                                                        head, tail_acc, partials, s, nseg, clk);              \
  else                                                                                                        \
    x16_launch<float, float, false, 1, false, false, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena,     \
                                                         ring, head, tail_acc, partials, s, nseg, clk);
    switch (h.x16_tune) {
      case 1: SEAS_X16_F32(1) break;
      case 2: SEAS_X16_F32(2) break;
      default: SEAS_X16_F32(0) break;
    }
#undef SEAS_X16_F32
    return;
  }
  // one variant: 16 windows; ensembles: BF16 with a BF16 rate history, or FP16 with
  // an FP32 one scaled per item; in the operator's tuned variant
#define SEAS_X16_ONE(TU)                                                                                      \
  if (bf) x16_launch<__bf16, float, false, 1, false, false, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, \
                                                                ring, head, tail_acc, partials, s, nseg, clk);  \
  else x16_launch<_Float16, float, true, 1, false, false, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, \
                                                              ring, head, tail_acc, partials, s, nseg, clk);
#define SEAS_X16_ENS(NT, TU)                                                                                  \
  if (bf) x16_launch<__bf16, __bf16, false, NT, true, false, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, \
                                                                 ring, head, tail_acc, partials, s, nseg, clk); \
  else x16_launch<_Float16, float, true, NT, false, false, TU>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, \
                                                               ring, head, tail_acc, partials, s, nseg, clk);
#define SEAS_X16_TUNED(TU)                   \
  if (h.n_variants == 1) {                   \
    SEAS_X16_ONE(TU)                         \
  } else {                                   \
    switch (h.ncols) {                       \
      case 16: SEAS_X16_ENS(1, TU) break;    \
      case 32: SEAS_X16_ENS(2, TU) break;    \
      case 64: SEAS_X16_ENS(4, TU) break;    \
      default: break;                        \
    }                                        \
  }
  switch (h.x16_tune) {
    case 1: SEAS_X16_TUNED(1) break;
    case 2: SEAS_X16_TUNED(2) break;
    default: SEAS_X16_TUNED(0) break;
  }
#undef SEAS_X16_TUNED
#undef SEAS_X16_ENS
#undef SEAS_X16_ONE
}

void launch_hmat_seg32(const HostOp& h, const void* items, const int32_t* seg_ptr, const int32_t* lagT,
                       const int32_t* lagCol, const int32_t* lagColOff, const float* arena, const void* ring,
                       bool ring_f64, int64_t head, const double* tail_acc, float* partials, hipStream_t s,
                       const int64_t* clk) {
  const int nseg = (int)h.seg_ptr3.size() - 1;
  if (nseg < 1) return;
#define SEAS_SEG32(NT)                                                                                         \
  if (ring_f64) x16_launch<float, double, false, NT>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, ring, head, \
                                                      tail_acc, partials, s, nseg, clk);                             \
  else x16_launch<float, float, false, NT>(h, items, seg_ptr, lagT, lagCol, lagColOff, arena, ring, head, tail_acc, \
                                           partials, s, nseg, clk);
  switch (h.ncols) {
    case 16: SEAS_SEG32(1) break;
    case 32: SEAS_SEG32(2) break;
    case 64: SEAS_SEG32(4) break;
    default: break;
  }
#undef SEAS_SEG32
}

}  // namespace seas
