// Device-side structures shared by the kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace seas {

struct SelfMode {      // one retained mode of one fault
  int fault, n, W;     // fault index, mode number (1..), window W_n
  int pad;
  int64_t tab;         // offset of K_n^T, T = 0..W_n
  int64_t ring;        // offset of the mode's coefficient ring (W_n entries)
};

struct SelfFaultDev {
  int off, Np, M, nm;  // first element, elements, 2 Np, retained modes
  int mode_off;        // first global mode index
  int tw;              // offset of the fault's twiddle table (M entries)
  double cfac;         // mu cs pi / (2 L)
};

struct Friction {
  const double *a, *b, *Dc, *sn, *V0, *f0, *eps;
};

// Arguments of the element kernels (predictor, corrector, prescribed output).
// Per-element arrays hold nv variants, variant-major ([nv][N]); the rate rings
// are [R][nv][N], the modal arrays [nv][n_modes], the coefficient rings
// [nv][dring_len] and the expired-slip accumulators [nv][tail_len].
template <typename TF>
struct StepArgs {
  int N, nv, n_modes;
  int64_t tail_len, dring_len;
  double dt, eta, t_next;
  double dts;               // length of this step: dt (the grid step) times gamma
  int64_t gamma;            // grid steps in this step (1: the fixed step)
  const int* fault_of;
  const SelfFaultDev* sf;
  const double2* tw;
  const double2* F;          // modal stress of the current stage
  const double* f_hist;      // interaction history part
  const int32_t *l0_ptr, *l0_col;
  const double* l0_val;
  const double *tau0, *tau0_rate;
  const int64_t* step0;     // per variant: the step at which its window started (tau0 loading time origin)
  Friction fric;
  double *V, *theta, *thdot, *delta;
  double *Vstar, *Vbar, *th2;
  double *f_self_out, *f_int_out;
  // per variant: Newton failure flag and the step index of the last committed step;
  // the corrector's results wait in V2/td2/fs2/fi2 (and the new slip coefficients in
  // Dnew) until the commit, which skips a failed variant
  int* fail;
  int64_t* good;
  double *V2, *td2, *fs2, *fi2;
  double2* Dnew;
  double2* dring;           // coefficient rings [nv][dring_len]
  const SelfMode* modes;
  int64_t self_head;        // time of the coefficient row the commit appends
  // history append (corrector)
  double* ring64;
  TF* ringop;               // operand copy (== ring64 for FP64 factors)
  int op_vfast;             // operand copy laid out [R][N][nv] (variant fastest; BF16 ensembles)
  int64_t R, time_new;      // ring length, time of the appended row
  // expired-slip accumulators
  double* tail_acc;
  const int32_t* tail_src;      // per source element: (accumulator, upper lag) entries (pairs of 2 ints)
  const int32_t* tail_src_ptr;  // per source element: range in tail_src
  int64_t first;            // earliest time held in the histories
  int tail;                 // static tail on
  int exact_state;          // state law integrated in closed form over the step (else explicit)
  // replays of a captured step sequence: the device-held step base is added to
  // time_new and self_head, and t_next = time_new dt (null: the values as given)
  const int64_t* clk;
};

void launch_hmat(const HostOp& h, int S, int n_items, const void* items, const int32_t* lagT, const int32_t* lagCol,
                 const int32_t* lagColOff, const void* arena, const void* ring, int64_t head,
                 const double* tail_acc, double* partials, int pstride, hipStream_t s,
                 const int64_t* clk = nullptr);
// far partials are FP32 when the far list runs on the matrix cores (FP32, S = 16)
bool far_partials_f32(const HostOp& h, int S);
void launch_reduce_far(const HostOp& h, int S, const void* partials, bool f32, const int32_t* ptr,
                       const int32_t* idx, double* f, hipStream_t s);
void launch_reduce_near(const HostOp& h, const double* partials, const int32_t* ptr, const int32_t* idx,
                        const double* base, double* f, hipStream_t s);
// zero one variant's rows of a [rows][nv][N] array of elem_bytes-sized values (elem_bytes even)
void launch_clear_variant(void* base, int64_t rows, int nv, int v, int N, int elem_bytes, hipStream_t s);
// far list on the matrix cores, one workgroup per segment: nseg segments from
// seg_ptr (a device pointer into the operator's segment offsets)
// (every launcher below that takes clk: a non-null clk holds a step base the
// kernel adds to its head / times, for replays of a captured step sequence)
void launch_hmat_x16(const HostOp& h, const void* items, const int32_t* seg_ptr, int nseg, const int32_t* lagT,
                     const int32_t* lagCol, const int32_t* lagColOff, const void* arena, const void* ring,
                     int64_t head, const double* tail_acc, float* partials, hipStream_t s,
                     const int64_t* clk = nullptr);
// ensembles: list 3 (FP32, segment layout) on the FP32 instance of the segment
// kernel, nv columns, staged from an FP32 (ring_f64 = false) or FP64 rate ring laid
// out [R][nv][N]; partials in list 0's buffer
void launch_hmat_seg32(const HostOp& h, const void* items, const int32_t* seg_ptr, const int32_t* lagT,
                       const int32_t* lagCol, const int32_t* lagColOff, const float* arena, const void* ring,
                       bool ring_f64, int64_t head, const double* tail_acc, float* partials, hipStream_t s,
                       const int64_t* clk = nullptr);
// FP32 far items of a 16-bit build (near-field blocks), S = 16 windows on the
// matrix cores, FP32 partials [p][16] in the 16-bit far list's partial buffer
void launch_hmat_f32far(const HostOp& h, int n_items, const void* items, const int32_t* lagT, const int32_t* lagCol,
                        const int32_t* lagColOff, const float* arena, const void* ring, int64_t head,
                        float* partials, hipStream_t s, const int64_t* clk = nullptr);
// self term over nv variants: modal arrays [nv][n_modes], rings [nv][dring_len], slip [nv][N]
void launch_self_hist(int n_modes, int nv, int64_t dring_len, const SelfMode* modes, const double* tab,
                      const double2* dring, int64_t time0, double2* Fh, hipStream_t s,
                      const int64_t* clk = nullptr);
// push: 1 stores the coefficients in the mode rings at push_time; Dsave (may be
// null) receives them instead, [nv][n_modes], for a later conditional push
void launch_dft(int n_modes, int nv, int N, int64_t dring_len, const SelfMode* modes, const SelfFaultDev* sf,
                const double* delta, const double* vel, double coef, const double2* tw, const double* tab,
                const double2* Fh, double2* Fout, double2* dring, int push, int64_t push_time, int64_t ring_head,
                hipStream_t s, double2* Dsave = nullptr, const int64_t* clk = nullptr);
// *clk = v (add = 0) or *clk += v (add = 1), one thread
void launch_clock(int64_t* clk, int64_t v, int add, hipStream_t s);
template <typename TF>
void launch_stage(const StepArgs<TF>& a, int stage, hipStream_t s);
// commit of a corrector: state, histories and outputs of every variant whose
// Newton solves of the step converged (a failed variant keeps its last good step)
template <typename TF>
void launch_commit(const StepArgs<TF>& a, hipStream_t s);
// Adaptive steps (a.gamma grid steps from n = a.time_new - a.gamma):
// per-block minima of xi Dc_e / V_e over ne values into part[0..nblocks)
void launch_dt_ev(const double* V, const double* Dc, int64_t ne, double xi, double* part, int nblocks, hipStream_t s);
// expired-slip accumulators at a long step's start: the committed rows that leave
// the windows, and its interior rows that do, at the starting rate V
template <typename TF>
void launch_tail_advance(const StepArgs<TF>& a, hipStream_t s);
// rate rows [lo, hi] (grid times) of every variant := src ([nv][N]), FP64 ring and operand copy
template <typename TF>
void launch_fill_rows(const StepArgs<TF>& a, int64_t lo, int64_t hi, const double* src, hipStream_t s);
// slip coefficients of a long step's interior grid times on the line from D^n to
// Dend ([nv][n_modes]); commit = 0 also keeps D^n in Dsv first (the ring slot of
// D^n may be among those written), commit = 1 takes D^n from Dsv
void launch_fill_modes(int n_modes, int nv, int64_t dring_len, const SelfMode* modes, double2* dring, int64_t n,
                       int64_t gamma, const double2* Dend, double2* Dsv, int commit, hipStream_t s);
template <typename TF>
void launch_prescribed_push(const StepArgs<TF>& a, const double* Vin, hipStream_t s);
template <typename TF>
void launch_prescribed_out(const StepArgs<TF>& a, const double* Vprev, double* fout, hipStream_t s);

}  // namespace seas
