// Internal declarations of the stress-transfer library (host and device).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "seas.h"

namespace seas {

struct Error : std::runtime_error {
  seas_status code;
  Error(seas_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ---------------------------------------------------------------- geometry
struct Fault {
  double cx, cy, nx, ny;  // centroid, unit normal e2'
  double tx, ty;          // tangent e1' = e3 x e2' = (-ny, nx)
  double L, dx;           // length, element size
  int Np, off;            // elements, global index of the first one
  double midx(int j) const { return cx + (-0.5 * L + (j + 0.5) * dx) * tx; }
  double midy(int j) const { return cy + (-0.5 * L + (j + 0.5) * dx) * ty; }
};

// ---------------------------------------------------------------- device work items
// One work item of the per-step interaction evaluation: a run of lags of one
// H-matrix block, all low-rank or all dense, whose factors are contiguous in the
// factor arena starting at `data`.
//   low rank (kind 0): W panel [q][ncol] (column fastest), then U panel [ncol][p]
//   dense    (kind 1): [nlag][q][p] (row fastest)
// The history row of lag T is the ring slot of time (head - T); src = 1 marks the
// static-tail item whose single "history row" is the expired-slip accumulator of
// its pair (at tail_off).
struct Item {
  int64_t data;      // element offset in the factor arena
  int32_t kind;      // 0 low rank, 1 dense
  int32_t src;       // 0 ring, 1 tail accumulator
  int32_t p, q;      // block rows (receivers) and columns (sources)
  int32_t row0;      // global receiver index of the block's first row
  int32_t col0;      // global source index of the block's first column
  int32_t nlag;      // lags in this item
  int32_t lag_off;   // offset in the lag arrays (T values; column prefix for low rank)
  int32_t ncol;      // total rank columns (low rank)
  int32_t part;      // offset of this item's p partial sums
  int32_t tail_off;  // offset of the pair's accumulator (src = 1)
  float scale;       // 16-bit factors: stored values times scale are the factors (1 otherwise)
};
static_assert(sizeof(Item) == 56, "Item layout");

constexpr int kItemThreads = 256;
constexpr int kDtEvBlocks = 1024;  // blocks of the adaptive step rule's minimum
constexpr int kHistMax = 6144;   // history values staged in LDS per item: (span of lags + S - 1) * q
constexpr int kColMax = 1024;    // low-rank columns (and lags) per item
constexpr int kZMax = 2048;      // low-rank columns times steps per item
constexpr int kMaxTimeBlock = 32;
constexpr int kTuneVariants = 3;  // variants of the FP32 one-variant segment kernel
// 16-bit factors (the matrix-core path): rows padded to 8 values (16 B)
constexpr int kHist16 = 16384;   // 16-bit history values staged per item: span * variants * q8
// ensemble products of 32 or more columns run two workgroups per CU (registers),
// so they stage twice the history per item; one variant's 32 time windows keep
// the 16-column budget (four workgroups per CU)
inline bool seg_wide(int ncols, int nv) { return ncols >= 32 && nv > 1; }
inline int hist16_limit(int ncols, int nv) { return seg_wide(ncols, nv) ? 2 * kHist16 : kHist16; }
constexpr int kZ16 = 4096;       // 16-bit projected values per low-rank item: ncol8 * columns
// (the end of the kernel's buffer holds the staging maxima: one per wave, or
// one per variant for scaled ensemble panels, 2 x 16 or 2 x 64 16-bit slots)
inline int z16_limit(int ncols, int nv) { return seg_wide(ncols, nv) ? 2 * kZ16 - 128 : kZ16 - 32; }
constexpr int kMaxVariants = 64;
constexpr int64_t kSegElems = 1 << 19;  // 16-bit factor values per segment (one workgroup; 1 MiB)
inline int round8(int x) { return (x + 7) & ~7; }
// LDS row stride of a staged 16-bit panel row of q8 values: an odd number of
// 16-byte groups, so that the 16 rows one MFMA operand reads fall in distinct banks
inline int ld16(int q8) { return ((q8 >> 3) & 1) ? q8 : q8 + 8; }
// rows of a multi-item segment: its accumulators stay in registers
inline int seg_rows_max(int ncols) { return ncols == 16 ? 512 : 256; }
// Segment far list (matrix-core kernel) with eb bytes per stored value: 2 for
// BF16 / FP16, 4 for FP32 (16 windows of one variant, or the FP32 list of FP16
// ensembles). The FP32 form stages the
// same LDS bytes as the 16-bit one, so half as many values.
inline int seg_hist_limit(int ncols, int eb, int nv) {
  return eb == 2 ? hist16_limit(ncols, nv) : hist16_limit(ncols, nv) / 2;
}
inline int seg_z_limit(int ncols, int eb, int nv) {
  return eb == 2 ? z16_limit(ncols, nv) : (seg_wide(ncols, nv) ? 2 * kZ16 : kZ16) / 2 - 4;
}
// ensembles: lags below this of admissible blocks, every lag of near-field
// blocks and the static tail are kept in FP32 (list 3)
constexpr int kEnsSplit = 16;
// LDS row stride of q8 staged values: an odd number of 16-byte groups
inline int seg_ld(int q8, int eb) {
  const int g = 16 / eb;
  return ((q8 / g) & 1) ? q8 : q8 + g;
}

// ---------------------------------------------------------------- host operator
struct PairWin {
  int a, b, T_init, T_end;
  int img = 0;  // 1: the source is the mirror image of fault b (free surface); its kernel enters with sign -1
};

struct BlockDesc {
  int pair, a, b, r0, r1, s0, s1, adm;
  int T_end;      // upper lag of the block (the pair's, or its own with cluster_windows)
  int tail_base;  // first expired-slip accumulator of the block's source columns (its own or the pair's)
};

struct SelfFault {          // self-term tables of one fault
  int Np, M, nm;            // elements, padded length, retained modes
  int mode_off;             // global offset of this fault's modes (1..nm)
  std::vector<int> W;       // W_n, n = 1..nm
  int tail = 0;             // 1: the table's entry W_n + 1 is the static tail R_n
  std::vector<int64_t> tab_off;   // offset of K_n^T (T = 0..W_n + tail) in the table
  std::vector<int64_t> ring_off;  // offset of the D ring of mode n (length W_n + tail)
  double cfac;              // mu cs pi / (2 L): F_n = -cfac * n * sum K_n^T D
};

struct HostOp {
  seas_params_t prm;
  std::vector<Fault> faults;
  // free surface: the mirror image of each fault across the surface line, its
  // elements in the order of the original's (same offsets into the rate history)
  std::vector<Fault> images;
  int N = 0;
  double dt = 0, eta = 0;
  std::vector<PairWin> pairs;
  std::vector<std::vector<BlockDesc>> blocks;  // per pair
  // work items: list 0 applied once per block of time_block steps (lags >= S, or
  // everything when S = 1), list 1 every step (lags 1..S-1 and the static tail)
  int time_block = 1;
  int n_variants = 1;                 // friction variants sharing the operator (ensemble columns)
  int ncols = 1;                      // columns of the far-list products: time_block * n_variants
  int x16_tune = 0;                   // variant of the FP32 one-variant segment kernel (seas_operator_tune)
  bool x16 = false;                   // far list in BF16/FP16 on the matrix cores, near list in FP32
  bool use_mfma = true;               // FP32, S = 16 far list on the matrix cores
  // far list in the segment layout of the matrix-core kernel (16-bit builds, and
  // FP32 builds with S = 16 unless SEAS_NO_SEG is set); near list then in its own
  // FP32 arena
  bool seg = false;
  int seg_eb = 2;                     // bytes per stored value of the segment far list
  // list 2 (16-bit builds with one variant): the far lags of near-field (not
  // admissible) blocks, kept in FP32 and applied with list 0 by the FP32 matrix-core
  // pass; their partials share list 0's buffer and reduction lists
  // list 3 (ensembles, ens32): near-field blocks, lags below kEnsSplit of
  // admissible blocks and the static tail, in FP32 in the segment layout, applied
  // by the FP32 instance of the segment kernel (segments seg_ptr3, arena of
  // arena32s_elems values) on the FP32 history copy (FP16) or the FP64 history
  // (BF16, whose copy is BF16); partials and reduction lists shared with list 0
  std::vector<Item> items[4];
  std::vector<int32_t> lagT;          // nlag lag values per item (ascending)
  std::vector<int32_t> lagCol;        // nlag+1 column prefix per item
  std::vector<int32_t> lagColOff[4];  // per item: offset into lagCol
  // time-blocked builds (S > 1): the far items whose lags lie in [S, 2S) (block-start
  // items) come last in their list, in segments of their own; the rest (lags >= 2S)
  // reads only history that is complete when the previous time block starts, so it
  // can be applied while the previous block steps
  int64_t first_items[4] = {0, 0, 0, 0};  // block-start items at the end of items[L]
  int64_t first_segs = 0;                 // block-start segments at the end of seg_ptr
  bool ens32 = false;
  std::vector<int32_t> seg_ptr3;
  int64_t arena32s_elems = 0;
  int64_t arena_elems = 0;
  int64_t arena_near_elems = 0;       // segment operators: FP32 arena of the near list
  std::vector<int32_t> seg_ptr;       // segment operators: far items of each segment (workgroup)
  int64_t n_partials[2] = {0, 0};
  std::vector<int32_t> red_ptr[2];    // N+1 per list
  std::vector<int32_t> red_idx[2];    // base partial index of each (receiver, item)
  std::vector<int32_t> tail_off; // per pair: offset of its accumulator; total tail_len
  int64_t tail_len = 0;
  // expired-slip updates per source element (global index): CSR over (accumulator,
  // upper lag) entries, one per pair (or per block with cluster_windows) whose
  // source columns hold the element
  std::vector<int32_t> tail_src_ptr, tail_src;
  // lag-0 CSR (FP64)
  std::vector<int32_t> l0_ptr, l0_col;
  std::vector<double> l0_val;
  // self term
  std::vector<SelfFault> self;
  std::vector<double> self_tab;  // K_n^T, all faults
  int64_t self_ring_len = 0;     // complex entries over all rings
  int n_modes = 0;               // total modes over faults
  int max_lag = 0, max_self_W = 0, ring_len = 0;
  // stats
  int64_t dense_entries = 0, stored_entries = 0, self_entries = 0;
  double build_seconds = 0;
};

// Factor values per block, in block order, and each block's offsets in the arenas.
// F64 / F32 operators: one arena (f64 or f32, offsets `off`). Segment operators:
// the far list in f16 (bit patterns of BF16 or FP16) or f32s (FP32), offsets
// `off`, and the near list in f32 (offsets `off32`). Ensembles: list 3 in f32s
// (offsets `off3`).
struct HostFactors {
  std::vector<std::vector<double>> f64;
  std::vector<std::vector<float>> f32;
  std::vector<std::vector<uint16_t>> f16;
  std::vector<std::vector<float>> f32s;
  std::vector<int64_t> off, off32, off3;
};

// message returned by seas_last_error() on the calling thread (api.hip)
void set_last_error(const std::string& msg);

// host build (build.cpp)
void build_host(const seas_fault_t* f, int nf, const seas_params_t& prm, HostOp& op, HostFactors& hf);
uint16_t to_bf16(float x);
uint16_t to_f16(float x);
float from_bf16(uint16_t b);
float from_f16(uint16_t b);

double kernel_entry(const Fault& A, int i, const Fault& B, int j, int T, double dt, double cs);
double static_stress(const Fault& A, int i, const Fault& B, int j, double mu);
void self_cells(int n, int W, double dt, double L, double cs, double* out);

}  // namespace seas
