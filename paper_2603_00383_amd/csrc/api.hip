// C ABI of the stress-transfer library: operator upload, state management and
// the per-step launch sequence. See include/seas.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace seas;

namespace {

thread_local std::string g_err;

#define HIPCHK(x)                                                                                       \
  do {                                                                                                  \
    hipError_t e_ = (x);                                                                                \
    if (e_ != hipSuccess) throw Error(SEAS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));    \
  } while (0)

template <typename F>
seas_status guard(F&& f) {
  try {
    f();
    return SEAS_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return SEAS_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return SEAS_ERR_INTERNAL;
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

void* dalloc(std::vector<DevBuf>& owned, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(SEAS_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  owned.push_back({p, bytes});
  return p;
}

template <typename T>
T* upload(std::vector<DevBuf>& owned, const std::vector<T>& v) {
  T* d = (T*)dalloc(owned, v.size() * sizeof(T));
  if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// Partial sums of seas_eval_prescribed_noalloc: a fixed device array, one copy per
// GPU for the life of the process. Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current); host code uses only
// that address, never the array's name.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) throw Error(SEAS_ERR_INVALID_ARG, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(SEAS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

double host_state_rate(double V, double th, double Dc, double eps) {
  const double r = V * th / Dc;
  if (eps == 1.0) return 1.0 - r;
  return (std::pow(r, -eps) - 1.0) * r / eps;
}

}  // namespace

void seas::set_last_error(const std::string& msg) { g_err = msg; }

struct seas_op {
  HostOp h;
  int device = 0;
  std::vector<DevBuf> owned;
  void* arena = nullptr;
  float* arena_near = nullptr;  // 16-bit operators: FP32 near-list factors
  int32_t* seg_ptr = nullptr;   // 16-bit operators: far-list segments
  Item* items[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t *lagT = nullptr, *lagCol = nullptr, *lagColOff[4] = {nullptr, nullptr, nullptr, nullptr};
  float* arena32s = nullptr;    // FP16 ensembles: FP32 segment list (list 3)
  int32_t* seg_ptr3 = nullptr;
  int32_t *red_ptr[2] = {nullptr, nullptr}, *red_idx[2] = {nullptr, nullptr};
  int32_t *l0_ptr = nullptr, *l0_col = nullptr;
  double* l0_val = nullptr;
  SelfMode* modes = nullptr;
  SelfFaultDev* sf = nullptr;
  double2* tw = nullptr;
  double* tab = nullptr;
  int* fault_of = nullptr;
  int32_t *tail_src = nullptr, *tail_src_ptr = nullptr;
  std::vector<SelfMode> hmodes;
  std::vector<SelfFaultDev> hsf;
  size_t elem_bytes = 8;  // bytes of a stored far-list factor value
  size_t ring_bytes = 8;  // bytes of a value of the rate history's operand copy (8: the FP64 ring itself)
  bool host_only = false;
  HostFactors hf;         // host factors (host_only)
  ~seas_op() {
    for (auto& b : owned) (void)hipFree(b.p);
  }
};

struct seas_state {
  seas_op* op = nullptr;
  int nv = 1;    // variants
  int mode = 0;  // 0 fresh, 1 prescribed, 2 stepping
  int64_t step = 0, first = 0;
  std::vector<DevBuf> owned;
  std::vector<DevBuf> ckpt;  // buffers that make up the state
  double *V, *theta, *thdot, *delta, *tau0, *tau0_rate;
  double *fa, *fb, *fDc, *fsn, *fV0, *ff0, *feps;
  double *Vstar, *Vbar, *th2, *f_hist, *f_self, *f_int;
  int64_t* step0;  // per variant: step at which its window started
  double* ring64;
  void* ringop;
  double* tail_acc;
  void* partials_far;      // FP64, or FP32 when the far list runs on the matrix cores
  double* partials_near;
  double* f_far;             // far part of the interaction for the S evaluations of a time block
  int64_t block_head = INT64_MIN / 2;  // head at which f_far was computed
  // adaptive steps: steps taken, gamma of the last one, per-block minima of the
  // step rule (device) and the slip coefficients at a long step's start
  int64_t steps_taken = 0, last_gamma = 1;
  int64_t gamma_cap = 0;  // > 0: this state's cap on gamma (below the operator's gamma_max)
  double* dtev = nullptr;
  double2* Dsv = nullptr;
  int run_S = 0;                        // 1: far list applied every step (plain form); else the build's S
  double2 *dring, *Fh, *F;
  int* fail;                 // per variant: a Newton solve failed (state held at its last good step)
  int64_t* good;             // per variant: step index of the last committed step
  double *V2, *td2, *fs2, *fi2;  // corrector results awaiting the commit
  double2* Dnew;             // corrector slip coefficients awaiting the commit
  bool timing = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  size_t n_ev = 0;             // pairs recorded since the last read
  // second stream of a step (default priority): the self history and the
  // predictor transform run there beside the interaction history part
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // block lookahead (time-blocked builds): the far items with lags >= 2S of the
  // next time block run on their own stream (default priority) while the current
  // block steps; la_head is the block head whose share is in flight there (only
  // within one seas_state_step call, which always consumes it)
  bool overlap = true;
  hipStream_t la = nullptr;
  hipEvent_t ev_la_go = nullptr, ev_la_done = nullptr;
  int64_t la_head = INT64_MIN / 2;
  // captured steps (seas_state_set_graph): one graph of g_unit steps that starts at
  // a time-block start, captured with step times relative to 0 on the capture
  // stream and replayed on the caller's stream; its kernels add the step base
  // *clk, which the graph's last node advances by g_unit
  bool graph = false, capturing = false;
  int64_t* clk = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_unit = 0, g_runS = -1;
  int64_t g_replays = 0;
  ~seas_state() {
    if (side) (void)hipStreamSynchronize(side);
    if (la) (void)hipStreamSynchronize(la);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap) (void)hipStreamDestroy(cap);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_la_go) (void)hipEventDestroy(ev_la_go);
    if (ev_la_done) (void)hipEventDestroy(ev_la_done);
    if (side) (void)hipStreamDestroy(side);
    if (la) (void)hipStreamDestroy(la);
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto& b : owned) (void)hipFree(b.p);
  }
};

namespace {

// step base of the kernels being recorded: only while a step sequence is captured
inline const int64_t* clk_of(const seas_state* st) { return st->capturing ? st->clk : nullptr; }

template <typename TF>
StepArgs<TF> make_args(seas_op* op, seas_state* st) {
  const HostOp& h = op->h;
  StepArgs<TF> a{};
  a.N = h.N;
  a.nv = st->nv;
  a.n_modes = h.n_modes;
  a.tail_len = h.tail_len;
  a.dring_len = h.self_ring_len;
  a.dt = h.dt;
  a.eta = h.eta;
  a.fault_of = op->fault_of;
  a.sf = op->sf;
  a.tw = op->tw;
  a.F = st->F;
  a.f_hist = st->f_hist;
  a.l0_ptr = op->l0_ptr;
  a.l0_col = op->l0_col;
  a.l0_val = op->l0_val;
  a.tau0 = st->tau0;
  a.tau0_rate = st->tau0_rate;
  a.step0 = st->step0;
  a.fric = Friction{st->fa, st->fb, st->fDc, st->fsn, st->fV0, st->ff0, st->feps};
  a.V = st->V;
  a.theta = st->theta;
  a.thdot = st->thdot;
  a.delta = st->delta;
  a.Vstar = st->Vstar;
  a.Vbar = st->Vbar;
  a.th2 = st->th2;
  a.f_self_out = st->f_self;
  a.f_int_out = st->f_int;
  a.fail = st->fail;
  a.good = st->good;
  a.V2 = st->V2;
  a.td2 = st->td2;
  a.fs2 = st->fs2;
  a.fi2 = st->fi2;
  a.Dnew = st->Dnew;
  a.dring = st->dring;
  a.modes = op->modes;
  a.ring64 = st->ring64;
  a.ringop = (TF*)st->ringop;
  a.op_vfast = op->ring_bytes == 2;
  a.R = h.ring_len;
  a.tail_acc = st->tail_acc;
  a.tail_src = op->tail_src;
  a.tail_src_ptr = op->tail_src_ptr;
  a.first = st->first;
  a.tail = h.prm.int_tail;
  a.exact_state = h.prm.state_update == 1;
  a.dts = h.dt;
  a.gamma = 1;
  a.clk = clk_of(st);
  return a;
}

void record_start(seas_state* st, hipStream_t s) {
  if (!st->timing) return;
  if (st->ev.size() < 2 * (st->n_ev + 1)) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    st->ev.push_back(a);
    st->ev.push_back(b);
  }
  HIPCHK(hipEventRecord(st->ev[2 * st->n_ev], s));
}

void record_stop(seas_state* st, hipStream_t s) {
  if (!st->timing) return;
  HIPCHK(hipEventRecord(st->ev[2 * st->n_ev + 1], s));
  st->n_ev++;
}

// Byte offset of the near partials and total bytes when both partial buffers of
// one evaluation share one allocation (far: FP32 on the matrix-core segment
// path, else FP64; near: FP64), the near ones 256-byte aligned.
std::pair<size_t, size_t> partial_layout(const HostOp& h) {
  const size_t far = (size_t)h.n_partials[0] * (h.seg ? 4 : 8);
  const size_t near_off = (far + 255) & ~(size_t)255;
  return {near_off, near_off + (size_t)h.n_partials[1] * 8};
}

// Far lists, or one part of them, for the S windows starting at `head`: all items
// (kFarAll), the items with lags >= 2S (kFarRest) or the block-start items with
// lags in [S, 2S) (kFarFirst); the parts write disjoint partial sums.
enum FarPart { kFarAll, kFarRest, kFarFirst };

void launch_far(seas_op* op, seas_state* st, int64_t head, FarPart part, int Sl, void* pfar, hipStream_t s) {
  const HostOp& h = op->h;
  // [a, b) of a list of n entries whose last nfirst are block-start ones
  auto range = [&](int64_t n, int64_t nfirst, int64_t& a, int64_t& b) {
    a = part == kFarFirst ? n - nfirst : 0;
    b = part == kFarRest ? n - nfirst : n;
  };
  int64_t a, b;
  if (h.seg) {
    range((int64_t)h.seg_ptr.size() - 1, h.first_segs, a, b);
    launch_hmat_x16(h, op->items[0], op->seg_ptr + a, (int)(b - a), op->lagT, op->lagCol, op->lagColOff[0],
                    op->arena, st->ringop, head, st->tail_acc, (float*)pfar, s, clk_of(st));
    range((int64_t)h.items[2].size(), h.first_items[2], a, b);
    launch_hmat_f32far(h, (int)(b - a), op->items[2] + a, op->lagT, op->lagCol, op->lagColOff[2] + a,
                       op->arena_near, st->ringop, head, (float*)pfar, s, clk_of(st));
    if (h.ens32 && part == kFarAll) {
      // BF16 ensembles keep a BF16 history copy: their FP32 list reads the FP64 history
      const bool r64 = op->ring_bytes == 2;
      launch_hmat_seg32(h, op->items[3], op->seg_ptr3, op->lagT, op->lagCol, op->lagColOff[3], op->arena32s,
                        r64 ? (const void*)st->ring64 : (const void*)st->ringop, r64, head, st->tail_acc,
                        (float*)pfar, s, clk_of(st));
    }
  } else {
    range((int64_t)h.items[0].size(), h.first_items[0], a, b);
    launch_hmat(h, Sl, (int)(b - a), op->items[0] + a, op->lagT, op->lagCol, op->lagColOff[0] + a, op->arena,
                st->ringop, head, st->tail_acc, (double*)pfar, h.time_block, s, clk_of(st));
  }
}

// Block lookahead of one step: `next` asks for the next block's far items with
// lags >= 2S to be launched on the lookahead stream when this step starts a block.
struct Lookahead {
  bool next;
};

// Interaction history part at `head` into st->f_hist. The far list is applied
// once per time block (S windows: heads block_head .. block_head + S - 1), the
// near list (lags 1..S-1 and the static tail) at every head. In the plain form
// (S = 1, or run_S = 1) the far list is applied at every head. Time-blocked:
// the items with lags >= 2S read history rows up to head - S - 1 only, so with a
// lookahead (`la`) they are launched for the next block on the lookahead stream as
// soon as this block's far sums are reduced, and the next block start waits for
// them and applies its block-start items (lags [S, 2S)) alone.
void eval_history(seas_op* op, seas_state* st, int64_t head, hipStream_t s, void* pfar = nullptr,
                  double* pnear = nullptr, const Lookahead* la = nullptr) {
  const HostOp& h = op->h;
  // partial sums: the state's buffers unless the caller brings its own
  if (!pfar) pfar = st->partials_far;
  if (!pnear) pnear = st->partials_near;
  const int S = h.time_block;
  const int nnear = (int)h.items[1].size();
  const bool plain = S == 1 || st->run_S == 1;
  int64_t k = head - st->block_head;
  if (plain || k < 0 || k >= S) {
    // plain form on a time-blocked build: window 0 of the far list at this head
    // (the segment kernel always forms its S windows; the plain form uses window 0)
    const int Sl = (plain && !h.seg) ? 1 : S;
    if (plain) {
      record_start(st, s);
      launch_far(op, st, head, kFarAll, Sl, pfar, s);
      record_stop(st, s);
    } else {
      // the timed launch is the part with lags >= 2S (most of the far list)
      if (la && st->la_head == head) {
        HIPCHK(hipStreamWaitEvent(s, st->ev_la_done, 0));
      } else {
        record_start(st, s);
        launch_far(op, st, head, kFarRest, Sl, pfar, s);
        record_stop(st, s);
      }
      launch_far(op, st, head, kFarFirst, Sl, pfar, s);
    }
    st->la_head = INT64_MIN / 2;
    const bool f32p = far_partials_f32(h, Sl);
    launch_reduce_far(h, h.seg ? h.ncols : Sl, pfar, f32p, op->red_ptr[0], op->red_idx[0],
                      nnear == 0 ? st->f_hist : st->f_far, s);
    if (la && la->next && !plain) {
      // the partial sums are free again once the reduction has read them
      HIPCHK(hipEventRecord(st->ev_la_go, s));
      HIPCHK(hipStreamWaitEvent(st->la, st->ev_la_go, 0));
      record_start(st, st->la);
      launch_far(op, st, head + S, kFarRest, Sl, pfar, st->la);
      record_stop(st, st->la);
      HIPCHK(hipEventRecord(st->ev_la_done, st->la));
      st->la_head = head + S;
    }
    if (nnear == 0) return;
    st->block_head = plain ? INT64_MIN / 2 : head;
    k = 0;
  }
  const void* arena_near = h.seg ? (const void*)op->arena_near : op->arena;
  launch_hmat(h, 1, nnear, op->items[1], op->lagT, op->lagCol, op->lagColOff[1], arena_near, st->ringop, head,
              st->tail_acc, pnear, 1, s, clk_of(st));
  launch_reduce_near(h, pnear, op->red_ptr[1], op->red_idx[1], st->f_far + k * h.N, st->f_hist, s);
}

// Adaptive steps (Section 2.4.1, step 1): gamma = ceil(min xi Dc / V / dt) over
// every element and variant, at least 1, at most gamma_max (read back to the host:
// the evaluation heads depend on it).
int64_t choose_gamma(seas_op* op, seas_state* st, hipStream_t s) {
  const HostOp& h = op->h;
  const int64_t ne = (int64_t)h.N * st->nv;
  const int nb = (int)std::min<int64_t>(kDtEvBlocks, (ne + 255) / 256);
  const double xi = h.prm.adapt_xi > 0.0 ? h.prm.adapt_xi : 0.5;
  launch_dt_ev(st->V, st->fDc, ne, xi, st->dtev, nb, s);
  double part[kDtEvBlocks];
  HIPCHK(hipMemcpyAsync(part, st->dtev, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double m = part[0];
  for (int b = 1; b < nb; ++b) m = std::min(m, part[b]);
  int64_t gmax = h.prm.gamma_max > 0 ? h.prm.gamma_max : (int64_t)1 << 20;
  if (st->gamma_cap > 0) gmax = std::min(gmax, st->gamma_cap);
  if (!(m > 0.0)) return 1;  // a rate that is not finite and positive: the solve reports it
  const double q = std::ceil(m / h.dt);
  return q >= (double)gmax ? gmax : std::max<int64_t>(1, (int64_t)q);
}

// One step of gamma > 1 grid steps from n: the rate and slip histories stay on the
// grid. The step's interior intervals n+1 .. n+gamma-1 enter its history sums at the
// starting rate V^n and the interior slip coefficients at the line from D^n to D*;
// the commit gives the interior rows the averaged rate and the coefficients the
// line to D** (the oracle's SeasState.step states the same). Rows and coefficients
// older than the windows need not be written: only the last ring_len - 2 rows and
// W_n coefficients of a mode can be read again.
template <typename TF>
void do_long_step(seas_op* op, seas_state* st, int64_t g, hipStream_t s) {
  const HostOp& h = op->h;
  const int nm = h.n_modes, nv = st->nv;
  const int64_t dl = h.self_ring_len;
  const int64_t n = st->step;
  StepArgs<TF> a = make_args<TF>(op, st);
  a.gamma = g;
  a.dts = (double)g * h.dt;
  a.t_next = (double)(n + g) * h.dt;
  a.time_new = n + g;
  a.self_head = n + g;
  const int64_t lo = std::max<int64_t>(n + 1, n + g - h.ring_len + 2), hi = n + g - 1;
  if (a.tail) launch_tail_advance<TF>(a, s);          // before the interior rows overwrite old ones
  launch_fill_rows<TF>(a, lo, hi, st->V, s);
  // self term: D* (kept in Dnew), the interior coefficients, the history at n+gamma, F*
  launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, st->V, a.dts, op->tw, op->tab, nullptr, st->F, st->dring,
             0, 0, 0, s, st->Dnew);
  launch_fill_modes(nm, nv, dl, op->modes, st->dring, n, g, st->Dnew, st->Dsv, 0, s);
  launch_self_hist(nm, nv, dl, op->modes, op->tab, st->dring, n + g, st->Fh, s);
  launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, st->V, a.dts, op->tw, op->tab, st->Fh, st->F, st->dring,
             0, 0, 0, s);
  eval_history(op, st, n + g - 1, s);                 // interaction at t_{n+gamma}: lags >= 1 and the tail
  launch_stage<TF>(a, 0, s);
  launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, st->Vbar, a.dts, op->tw, op->tab, st->Fh, st->F,
             st->dring, 0, n + g, n + g, s, st->Dnew);
  launch_stage<TF>(a, 1, s);
  launch_commit<TF>(a, s);
  launch_fill_rows<TF>(a, lo, hi, st->Vbar, s);
  launch_fill_modes(nm, nv, dl, op->modes, st->dring, n, g, st->Dnew, st->Dsv, 1, s);
  st->step = n + g;
}

void ensure_side(seas_state* st) {
  if (st->side) return;
  HIPCHK(hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&st->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&st->ev_join, hipEventDisableTiming));
}

template <typename TF>
void step_loop(seas_op* op, seas_state* st, int n_steps, hipStream_t s) {
  const HostOp& h = op->h;
  const int nm = h.n_modes, nv = st->nv;
  const int64_t dl = h.self_ring_len;
  if (n_steps > 0) ensure_side(st);
  const int S = h.time_block;
  const bool la_on = st->overlap && S > 1 && st->run_S != 1;
  if (la_on && !st->la) {
    HIPCHK(hipStreamCreateWithFlags(&st->la, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&st->ev_la_go, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&st->ev_la_done, hipEventDisableTiming));
  }
  st->la_head = INT64_MIN / 2;
  for (int it = 0; it < n_steps; ++it) {
    const int64_t n = st->step;
    const int64_t g = h.prm.adaptive_dt ? choose_gamma(op, st, s) : 1;
    st->last_gamma = g;
    st->steps_taken++;
    if (g > 1) {
      do_long_step<TF>(op, st, g, s);
      continue;
    }
    // a lookahead is launched only for a block this call reaches, so the call
    // itself consumes every lookahead it starts
    const Lookahead la{it + S < n_steps};
    // The self history and the predictor transform read only what the previous
    // step left (coefficient rings, slip, rate) and write Fh and F, which the
    // interaction history part neither reads nor writes: they run on the side
    // stream from the step's start and rejoin before the predictor stage.
    HIPCHK(hipEventRecord(st->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(st->side, st->ev_fork, 0));
    launch_self_hist(nm, nv, dl, op->modes, op->tab, st->dring, n + 1, st->Fh, st->side, clk_of(st));
    launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, st->V, h.dt, op->tw, op->tab, st->Fh, st->F,
               st->dring, 0, 0, 0, st->side, nullptr, clk_of(st));
    HIPCHK(hipEventRecord(st->ev_join, st->side));
    eval_history(op, st, n, s, nullptr, nullptr, la_on ? &la : nullptr);
    HIPCHK(hipStreamWaitEvent(s, st->ev_join, 0));
    StepArgs<TF> a = make_args<TF>(op, st);
    a.t_next = (double)(n + 1) * h.dt;
    a.time_new = n + 1;
    a.self_head = n + 1;
    launch_stage<TF>(a, 0, s);
    // corrector: D** waits in Dnew; the commit appends it with the rest of the step
    // unless a solve of the variant failed
    launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, st->Vbar, h.dt, op->tw, op->tab, st->Fh, st->F,
               st->dring, 0, n + 1, n + 1, s, st->Dnew, clk_of(st));
    launch_stage<TF>(a, 1, s);
    launch_commit<TF>(a, s);
    st->step = n + 1;
  }
  st->la_head = INT64_MIN / 2;
  HIPCHK(hipGetLastError());
}

// Steps per captured graph when every step starts a time block (the plain form)
constexpr int kGraphPlainSteps = 16;

// Capture U fixed steps that start at a time-block start: recorded on the capture
// stream with step times 0 .. U-1 (the kernels add *clk), then a node that adds U
// to *clk. No block lookahead (it would reach into the next replay) and no timing
// events inside the graph.
template <typename TF>
void capture_steps(seas_op* op, seas_state* st, int U) {
  if (st->gexec) {
    HIPCHK(hipGraphExecDestroy(st->gexec));
    st->gexec = nullptr;
  }
  ensure_side(st);
  if (!st->cap) HIPCHK(hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
  const int64_t step = st->step, bh = st->block_head, taken = st->steps_taken, lg = st->last_gamma;
  const bool timing = st->timing, overlap = st->overlap;
  auto restore = [&] {
    st->step = step;
    st->block_head = bh;
    st->steps_taken = taken;
    st->last_gamma = lg;
    st->timing = timing;
    st->overlap = overlap;
    st->capturing = false;
  };
  st->step = 0;
  st->block_head = INT64_MIN / 2;
  st->timing = false;
  st->overlap = false;
  st->capturing = true;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal));
  try {
    step_loop<TF>(op, st, U, st->cap);
    launch_clock(st->clk, U, 1, st->cap);
  } catch (...) {
    (void)hipStreamEndCapture(st->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    restore();
    throw;
  }
  restore();
  HIPCHK(hipStreamEndCapture(st->cap, &g));
  const hipError_t e = hipGraphInstantiate(&st->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    st->gexec = nullptr;
    throw Error(SEAS_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
  }
  st->g_unit = U;
  st->g_runS = st->run_S;
}

// Fixed steps as replays of the captured graph where whole time blocks fit: eager
// steps up to the next block start, the replays, eager steps for the rest. Every
// step evaluates exactly as an eager one (same kernels, same values).
template <typename TF>
void do_steps(seas_op* op, seas_state* st, int n_steps, hipStream_t s) {
  const HostOp& h = op->h;
  if (!st->graph || h.prm.adaptive_dt) {
    step_loop<TF>(op, st, n_steps, s);
    return;
  }
  const int S = h.time_block;
  const bool plain = S == 1 || st->run_S == 1;
  const int U = plain ? kGraphPlainSteps : S;
  int done = 0;
  auto starts_block = [&] {
    const int64_t k = st->step - st->block_head;
    return plain || k < 0 || k >= S;
  };
  while (done < n_steps && !starts_block()) {
    step_loop<TF>(op, st, 1, s);
    ++done;
  }
  const int reps = (n_steps - done) / U;
  if (reps > 0) {
    if (!st->gexec || st->g_unit != U || st->g_runS != st->run_S) capture_steps<TF>(op, st, U);
    launch_clock(st->clk, st->step, 0, s);
    for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(st->gexec, s));
    st->step += (int64_t)reps * U;
    st->steps_taken += (int64_t)reps * U;
    st->last_gamma = 1;
    st->block_head = plain ? INT64_MIN / 2 : st->step - U;
    st->g_replays += reps;
    done += reps * U;
  }
  if (done < n_steps) step_loop<TF>(op, st, n_steps - done, s);
}

template <typename TF>
void do_prescribed(seas_op* op, seas_state* st, const double* V, int n_steps, double* f, hipStream_t s,
                   void* pfar = nullptr, double* pnear = nullptr) {
  const HostOp& h = op->h;
  const int nm = h.n_modes, nv = st->nv;
  const int64_t dl = h.self_ring_len;
  const size_t row = (size_t)h.N * nv;
  for (int it = 0; it < n_steps; ++it) {
    const int64_t n = st->step + 1;  // evaluating f^n
    const int64_t hd = n - 1;        // time of the newest rate, V^{n-1}
    StepArgs<TF> a = make_args<TF>(op, st);
    a.time_new = hd;
    // the accumulators of a new state already cover every time up to -T_end - 1 (the
    // window of the rate at time 0); re-pushing time 0 must not add that row again
    if (hd < 1) a.tail = 0;
    const double* Vrow = V + (size_t)it * row;
    launch_prescribed_push<TF>(a, Vrow, s);
    eval_history(op, st, hd, s, pfar, pnear);
    launch_self_hist(nm, nv, dl, op->modes, op->tab, st->dring, n, st->Fh, s);
    launch_dft(nm, nv, h.N, dl, op->modes, op->sf, st->delta, nullptr, 0.0, op->tw, op->tab, st->Fh, st->F,
               st->dring, 1, n, n, s);
    launch_prescribed_out<TF>(a, Vrow, f + (size_t)it * row, s);
    st->step = n;
  }
  HIPCHK(hipGetLastError());
}

// n values of the rate history's operand copy at element offset `off`, converted
// on the host; synchronises the stream (the conversion buffer is temporary).
void upload_op_seg(seas_op* op, void* ringop, size_t off, const double* row, size_t n, hipStream_t s) {
  if (op->ring_bytes == 8) return;
  if (op->ring_bytes == 4) {
    std::vector<float> v(row, row + n);
    HIPCHK(hipMemcpyAsync((float*)ringop + off, v.data(), n * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::vector<uint16_t> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = to_bf16((float)row[i]);
    HIPCHK(hipMemcpyAsync((uint16_t*)ringop + off, v.data(), n * 2, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
}

// One row (all variants, host layout [nv][N]) of the operand copy at ring slot
// `slot`; the BF16 ensemble copy is laid out [R][N][nv] (variant fastest).
void upload_op_row(seas_op* op, void* ringop, int64_t slot, const double* row, size_t n, hipStream_t s) {
  if (op->ring_bytes != 2) {
    upload_op_seg(op, ringop, (size_t)slot * n, row, n, s);
    return;
  }
  const size_t N = op->h.N, nv = n / N;
  std::vector<uint16_t> v(n);
  for (size_t k = 0; k < nv; ++k)
    for (size_t r = 0; r < N; ++r) v[r * nv + k] = to_bf16((float)row[k * N + r]);
  HIPCHK(hipMemcpyAsync((uint16_t*)ringop + (size_t)slot * n, v.data(), n * 2, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

// Variant v's N values of one ring slot of the BF16 ensemble copy ([R][N][nv]).
void upload_op_variant(seas_op* op, void* ringop, int64_t slot, int nv, int v, const double* x, hipStream_t s) {
  const size_t N = op->h.N;
  std::vector<uint16_t> b(N);
  for (size_t r = 0; r < N; ++r) b[r] = to_bf16((float)x[r]);
  HIPCHK(hipMemcpy2DAsync((uint16_t*)ringop + ((size_t)slot * N) * nv + v, (size_t)nv * 2, b.data(), 2, 2, N,
                          hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

seas_op* checked(seas_op* op) {
  if (!op) throw Error(SEAS_ERR_INVALID_ARG, "null operator");
  if (op->host_only) throw Error(SEAS_ERR_MISMATCH, "operator was built with host_only = 1");
  HIPCHK(hipSetDevice(op->device));
  return op;
}

}  // namespace

extern "C" {

const char* seas_last_error(void) { return g_err.c_str(); }
const char* seas_version(void) { return "seas-mi355x 0.2 (gfx950)"; }

double seas_round_factor(double x, int32_t factor_dtype) {
  switch (factor_dtype) {
    case SEAS_F32: return (double)(float)x;
    case SEAS_BF16: return (double)from_bf16(to_bf16((float)x));
    case SEAS_F16: return (double)from_f16(to_f16((float)x));
    default: return x;
  }
}

seas_status seas_build_operator(const seas_fault_t* faults, int32_t n_faults, const seas_params_t* params,
                                seas_op_t** out) {
  return guard([&] {
    if (!faults || !params || !out) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    auto op = std::make_unique<seas_op>();
    op->host_only = params->host_only != 0;
    if (!op->host_only) HIPCHK(hipGetDevice(&op->device));
    HostFactors& hf = op->hf;
    build_host(faults, n_faults, *params, op->h, hf);
    HostOp& h = op->h;
    const bool f32 = h.prm.factor_dtype == SEAS_F32;
    op->elem_bytes = h.x16 ? 2 : (f32 ? 4 : 8);
    // rate-history operand: FP32 (F16 stages it with a per-item scale; BF16 with one
    // variant converts it at staging), BF16 for BF16 ensembles (halves the history reads)
    op->ring_bytes = h.x16 ? ((h.n_variants > 1 && h.prm.factor_dtype == SEAS_BF16) ? 2 : 4) : op->elem_bytes;
    if (op->host_only) {
      *out = op.release();
      return;
    }
    // factor arenas, block by block
    op->arena = dalloc(op->owned, (size_t)h.arena_elems * op->elem_bytes);
    if (h.seg) op->arena_near = (float*)dalloc(op->owned, (size_t)h.arena_near_elems * 4);
    if (h.ens32) op->arena32s = (float*)dalloc(op->owned, (size_t)h.arena32s_elems * 4);
    for (size_t bi = 0; bi < hf.off.size(); ++bi) {
      const size_t n = h.x16 ? hf.f16[bi].size()
                             : (h.seg ? hf.f32s[bi].size() : (f32 ? hf.f32[bi].size() : hf.f64[bi].size()));
      const void* src = h.x16 ? (const void*)hf.f16[bi].data()
                              : (h.seg ? (const void*)hf.f32s[bi].data()
                                       : (f32 ? (const void*)hf.f32[bi].data() : (const void*)hf.f64[bi].data()));
      if (n > 0)
        HIPCHK(hipMemcpy((char*)op->arena + (size_t)hf.off[bi] * op->elem_bytes, src, n * op->elem_bytes,
                         hipMemcpyHostToDevice));
      if (h.seg && !hf.f32[bi].empty())
        HIPCHK(hipMemcpy(op->arena_near + hf.off32[bi], hf.f32[bi].data(), hf.f32[bi].size() * 4,
                         hipMemcpyHostToDevice));
      if (h.ens32 && !hf.f32s[bi].empty())
        HIPCHK(hipMemcpy(op->arena32s + hf.off3[bi], hf.f32s[bi].data(), hf.f32s[bi].size() * 4,
                         hipMemcpyHostToDevice));
      std::vector<double>().swap(hf.f64[bi]);
      std::vector<float>().swap(hf.f32[bi]);
      std::vector<uint16_t>().swap(hf.f16[bi]);
      std::vector<float>().swap(hf.f32s[bi]);
    }
    if (h.seg) op->seg_ptr = upload(op->owned, h.seg_ptr);
    if (h.ens32) op->seg_ptr3 = upload(op->owned, h.seg_ptr3);
    for (int L = 0; L < 4; ++L) {
      op->items[L] = upload(op->owned, h.items[L]);
      op->lagColOff[L] = upload(op->owned, h.lagColOff[L]);
    }
    for (int L = 0; L < 2; ++L) {
      op->red_ptr[L] = upload(op->owned, h.red_ptr[L]);
      op->red_idx[L] = upload(op->owned, h.red_idx[L]);
    }
    op->lagT = upload(op->owned, h.lagT);
    op->lagCol = upload(op->owned, h.lagCol);
    op->l0_ptr = upload(op->owned, h.l0_ptr);
    op->l0_col = upload(op->owned, h.l0_col);
    op->l0_val = upload(op->owned, h.l0_val);
    op->tab = upload(op->owned, h.self_tab);
    // self-term metadata and twiddle tables e^{-2 pi i k / M}
    std::vector<double2> tw;
    std::vector<int> fault_of(h.N);
    for (size_t k = 0; k < h.faults.size(); ++k) {
      const SelfFault& s = h.self[k];
      SelfFaultDev d;
      d.off = h.faults[k].off;
      d.Np = s.Np;
      d.M = s.M;
      d.nm = s.nm;
      d.mode_off = s.mode_off;
      d.tw = (int)tw.size();
      d.cfac = s.cfac;
      for (int e = 0; e < s.M; ++e) {
        const double ang = 2.0 * M_PI * (double)e / (double)s.M;
        tw.push_back(make_double2(std::cos(ang), -std::sin(ang)));
      }
      op->hsf.push_back(d);
      for (int n = 1; n <= s.nm; ++n) {
        SelfMode m;
        m.fault = (int)k;
        m.n = n;
        m.W = s.W[n - 1] + s.tail;  // the static tail is one more lag of the ring
        m.pad = 0;
        m.tab = s.tab_off[n - 1];
        m.ring = s.ring_off[n - 1];
        op->hmodes.push_back(m);
      }
      for (int j = 0; j < s.Np; ++j) fault_of[d.off + j] = (int)k;
    }
    op->sf = upload(op->owned, op->hsf);
    op->modes = upload(op->owned, op->hmodes);
    op->tw = upload(op->owned, tw);
    op->fault_of = upload(op->owned, fault_of);
    // expired-slip updates per source element
    op->tail_src = upload(op->owned, h.tail_src);
    op->tail_src_ptr = upload(op->owned, h.tail_src_ptr);
    *out = op.release();
  });
}

void seas_operator_destroy(seas_op_t* op) {
  if (op) {
    if (!op->host_only) (void)hipSetDevice(op->device);
    delete op;
  }
}

seas_status seas_operator_lag_matrix(const seas_op_t* op, int32_t a, int32_t b, int32_t T, double* out) {
  return guard([&] {
    if (!op || !out) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    if (!op->host_only) throw Error(SEAS_ERR_MISMATCH, "factors are only kept on the host with host_only = 1");
    const HostOp& h = op->h;
    const int nf = (int)h.faults.size();
    // b = nf + a: the pair of fault a with its own image (free surface), the only image
    // pair whose source columns no fault pair shares
    const bool own_img = !h.images.empty() && b == nf + a;
    if (a < 0 || b < 0 || a >= nf || (b >= nf && !own_img) || a == b || T < -1)
      throw Error(SEAS_ERR_INVALID_ARG, "bad pair/lag");
    const Fault &A = h.faults[a], &B = h.faults[own_img ? a : b];
    const int p_all = A.Np, q_all = B.Np;
    std::fill(out, out + (size_t)p_all * q_all, 0.0);
    if (T == 0) {
      for (int i = 0; i < p_all; ++i)
        for (int k = h.l0_ptr[A.off + i]; k < h.l0_ptr[A.off + i + 1]; ++k) {
          const int c = h.l0_col[k];
          if (c >= B.off && c < B.off + q_all) out[(size_t)i * q_all + (c - B.off)] = h.l0_val[k];
        }
      return;
    }
    // every item covering the pair adds its part: with a free surface the pair (a, b)
    // also holds the blocks of fault a against the image of b, on the same columns
    // the arenas are the concatenation of the per-block buffers: locate an element
    const HostFactors& hf = op->hf;
    auto elem_in = [&](const std::vector<int64_t>& off, int64_t e, int which) -> double {
      size_t lo = 0, hi = off.size();
      while (hi - lo > 1) {
        const size_t mid = (lo + hi) / 2;
        if (off[mid] <= e) lo = mid;
        else hi = mid;
      }
      while (lo + 1 < off.size() && off[lo + 1] == off[lo] &&
             (which == 3   ? hf.f32s[lo].empty()
              : which == 2 ? hf.f16[lo].empty()
              : which == 1 ? hf.f32[lo].empty()
                           : hf.f64[lo].empty()))
        ++lo;  // skip empty blocks that share the offset
      const int64_t k = e - off[lo];
      if (which == 3) return (double)hf.f32s[lo][k];
      if (which == 2)
        return h.prm.factor_dtype == SEAS_BF16 ? (double)from_bf16(hf.f16[lo][k]) : (double)from_f16(hf.f16[lo][k]);
      return which == 1 ? (double)hf.f32[lo][k] : hf.f64[lo][k];
    };
    for (int L = 0; L < 4; ++L)
    for (size_t ii = 0; ii < h.items[L].size(); ++ii) {
      const Item& it = h.items[L][ii];
      if (it.row0 < A.off || it.row0 >= A.off + p_all || it.col0 < B.off || it.col0 >= B.off + q_all) continue;
      const int ri = it.row0 - A.off, cj = it.col0 - B.off;
      const int32_t* cp = &h.lagCol[h.lagColOff[L][ii]];
      const bool sg = h.seg && (L == 0 || L == 3);
      const int which = sg ? ((h.x16 && L == 0) ? 2 : 3) : ((h.seg || h.prm.factor_dtype == SEAS_F32) ? 1 : 0);
      const std::vector<int64_t>& off = L == 3 ? hf.off3 : ((h.seg && L >= 1) ? hf.off32 : hf.off);
      auto elem = [&](int64_t e) { return elem_in(off, e, which); };
      for (int l = 0; l < it.nlag; ++l) {
        if (h.lagT[it.lag_off + l] != T) continue;
        if (sg) {
          const int q8 = round8(it.q), nc = it.ncol, nc8 = round8(nc);
          const double sc = it.scale;
          if (it.kind == 0) {
            for (int c = cp[l]; c < cp[l + 1]; ++c)
              for (int i = 0; i < it.p; ++i) {
                const double u = elem(it.data + (int64_t)nc * q8 + (int64_t)i * nc8 + c);
                for (int j = 0; j < it.q; ++j)
                  out[(size_t)(ri + i) * q_all + cj + j] += sc * u * elem(it.data + (int64_t)c * q8 + j);
              }
          } else {
            for (int i = 0; i < it.p; ++i)
              for (int j = 0; j < it.q; ++j)
                out[(size_t)(ri + i) * q_all + cj + j] +=
                    sc * elem(it.data + (int64_t)i * it.nlag * q8 + (int64_t)l * q8 + j);
          }
          continue;
        }
        if (it.kind == 0) {
          const int nc = it.ncol;
          for (int c = cp[l]; c < cp[l + 1]; ++c)
            for (int i = 0; i < it.p; ++i) {
              const double u = elem(it.data + (int64_t)it.q * nc + (int64_t)c * it.p + i);
              for (int j = 0; j < it.q; ++j)
                out[(size_t)(ri + i) * q_all + cj + j] += u * elem(it.data + (int64_t)j * nc + c);
            }
        } else {
          for (int j = 0; j < it.q; ++j)
            for (int i = 0; i < it.p; ++i)
              out[(size_t)(ri + i) * q_all + cj + j] += elem(it.data + ((int64_t)l * it.q + j) * it.p + i);
        }
      }
    }
  });
}

seas_status seas_operator_info(const seas_op_t* op, seas_op_info_t* out) {
  return guard([&] {
    if (!op || !out) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    const HostOp& h = op->h;
    std::memset(out, 0, sizeof(*out));
    out->n_faults = (int32_t)h.faults.size();
    out->n_elem = h.N;
    out->dt = h.dt;
    out->max_lag = h.max_lag;
    out->max_self_window = h.max_self_W;
    int64_t nb = 0;
    for (auto& v : h.blocks) nb += (int64_t)v.size();
    out->n_blocks = nb;
    out->n_items = (int64_t)h.items[0].size();
    out->n_items_near = (int64_t)h.items[1].size();
    out->time_block = h.time_block;
    int64_t far = 0, far32 = 0;
    for (const Item& it : h.items[0])
      far += it.kind == 0 ? (int64_t)it.ncol * (it.p + it.q) : (int64_t)it.nlag * it.p * it.q;
    for (int L = 2; L < 4; ++L)
      for (const Item& it : h.items[L])
        far32 += it.kind == 0 ? (int64_t)it.ncol * (it.p + it.q) : (int64_t)it.nlag * it.p * it.q;
    out->far_entries = far + far32;
    out->far_entries_f32 = far32;
    int64_t ff = 0, ff32 = 0;
    for (int L = 0; L < 3; L += 2) {
      const auto& its = h.items[L];
      for (size_t x = its.size() - (size_t)h.first_items[L]; x < its.size(); ++x) {
        const Item& it = its[x];
        const int64_t e = it.kind == 0 ? (int64_t)it.ncol * (it.p + it.q) : (int64_t)it.nlag * it.p * it.q;
        ff += e;
        if (L == 2) ff32 += e;
      }
    }
    out->far_entries_first = ff;
    out->far_entries_first_f32 = ff32;
    out->dense_entries = h.dense_entries;
    out->stored_entries = h.stored_entries;
    out->lag0_nnz = (int64_t)h.l0_val.size();
    out->self_entries = h.self_entries;
    out->bytes_per_step = (double)h.stored_entries * (double)op->elem_bytes + (double)h.self_entries * (8.0 + 16.0);
    out->flops_per_step = 2.0 * (double)h.stored_entries + 4.0 * (double)h.self_entries;
    out->build_seconds = h.build_seconds;
    out->factor_dtype = h.prm.factor_dtype;
    out->n_variants = h.n_variants;
    out->ncols = h.ncols;
    out->n_segments = h.seg ? (int64_t)h.seg_ptr.size() - 1 : 0;
    int64_t fb = 0;
    for (const Item& it : h.items[0]) {
      if (h.seg) {
        const int64_t q8 = round8(it.q);
        fb += h.seg_eb * (it.kind == 0 ? (int64_t)it.ncol * q8 + (int64_t)it.p * round8(it.ncol) : (int64_t)it.nlag * it.p * q8);
      } else {
        fb += (int64_t)op->elem_bytes *
              (it.kind == 0 ? (int64_t)it.ncol * (it.p + it.q) : (int64_t)it.nlag * it.p * it.q);
      }
    }
    for (const Item& it : h.items[2])
      fb += 4 * (it.kind == 0 ? (int64_t)it.ncol * (it.p + it.q) : (int64_t)it.nlag * it.p * it.q);
    for (const Item& it : h.items[3]) {
      const int64_t q8 = round8(it.q);
      fb += 4 * (it.kind == 0 ? (int64_t)it.ncol * q8 + (int64_t)it.p * round8(it.ncol) : (int64_t)it.nlag * it.p * q8);
    }
    out->far_bytes = fb;
    out->partial_bytes = (int64_t)partial_layout(h).second;
  });
}

seas_status seas_operator_windows(const seas_op_t* op, int32_t* T_init, int32_t* T_end) {
  return guard([&] {
    if (!op || !T_init || !T_end) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    size_t k = 0;
    for (const PairWin& w : op->h.pairs) {
      if (w.img) continue;  // the image pairs follow the fault pairs; see seas_operator_pair_window
      T_init[k] = w.T_init;
      T_end[k] = w.T_end;
      ++k;
    }
  });
}

// pair index of (a, b): b < nf the fault pair, b in [nf, 2 nf) the image of fault b - nf
static size_t pair_index(const HostOp& h, int32_t a, int32_t b) {
  const int nf = (int)h.faults.size();
  const bool img = b >= nf;
  const int bb = img ? b - nf : b;
  if (a < 0 || a >= nf || bb < 0 || bb >= nf || (a == bb && !img) || (img && h.images.empty()))
    throw Error(SEAS_ERR_INVALID_ARG, "bad pair");
  for (size_t pi = 0; pi < h.pairs.size(); ++pi)
    if (h.pairs[pi].a == a && h.pairs[pi].b == bb && h.pairs[pi].img == (img ? 1 : 0)) return pi;
  throw Error(SEAS_ERR_INTERNAL, "pair not found");
}

seas_status seas_operator_pair_window(const seas_op_t* op, int32_t a, int32_t b, int32_t* T_init, int32_t* T_end) {
  return guard([&] {
    if (!op || !T_init || !T_end) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    const PairWin& w = op->h.pairs[pair_index(op->h, a, b)];
    *T_init = w.T_init;
    *T_end = w.T_end;
  });
}

seas_status seas_operator_blocks(const seas_op_t* op, int32_t a, int32_t b, int32_t* blocks, int64_t* count) {
  return guard([&] {
    if (!op || !count) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    const HostOp& h = op->h;
    const auto& bl = h.blocks[pair_index(h, a, b)];
    if (blocks) {
      if (*count < (int64_t)bl.size()) throw Error(SEAS_ERR_INVALID_ARG, "block buffer too small");
      for (size_t i = 0; i < bl.size(); ++i) {
        blocks[6 * i + 0] = bl[i].r0;
        blocks[6 * i + 1] = bl[i].r1;
        blocks[6 * i + 2] = bl[i].s0;
        blocks[6 * i + 3] = bl[i].s1;
        blocks[6 * i + 4] = bl[i].adm;
        blocks[6 * i + 5] = bl[i].T_end;
      }
    }
    *count = (int64_t)bl.size();
  });
}

seas_status seas_operator_self_table(const seas_op_t* op, int32_t k, int32_t n, double* out, int32_t capacity,
                                     int32_t* W_n) {
  return guard([&] {
    if (!op || !W_n) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    const HostOp& h = op->h;
    if (k < 0 || k >= (int)h.self.size() || n < 1 || n > h.self[k].nm) throw Error(SEAS_ERR_INVALID_ARG, "bad mode");
    const SelfFault& s = h.self[k];
    *W_n = s.W[n - 1];
    if (out) {
      const int len = s.W[n - 1] + 1 + s.tail;
      if (capacity < len) throw Error(SEAS_ERR_INVALID_ARG, "capacity too small");
      std::memcpy(out, &h.self_tab[s.tab_off[n - 1]], sizeof(double) * len);
    }
  });
}

size_t seas_state_bytes(const seas_op_t* op, int32_t n_variants) {
  if (!op || n_variants < 1) return 0;
  const HostOp& h = op->h;
  const size_t N = (size_t)h.N * n_variants;
  size_t b = N * 8 * 23;                                         // per-element state and scratch
  b += (size_t)h.ring_len * N * 8;                               // FP64 rate history
  if (op->ring_bytes != 8) b += (size_t)h.ring_len * N * op->ring_bytes;  // operand copy
  b += (size_t)h.tail_len * 8 * n_variants;
  b += (size_t)h.n_partials[0] * (h.seg ? 4 : 8) + (size_t)h.n_partials[1] * 8;
  b += (size_t)h.time_block * N * 8;
  b += (size_t)h.self_ring_len * 16 * n_variants + (size_t)h.n_modes * 16 * 3 * n_variants;
  b += (size_t)n_variants * (sizeof(int) + sizeof(int64_t));
  return b;
}

seas_status seas_state_create(seas_op_t* op, int32_t n_variants, const seas_friction_t* fric, const double* V_init,
                              const double* theta_init, const double* tau0, const double* tau0_rate,
                              const double* delta_init, void* stream, seas_state_t** out) {
  return guard([&] {
    checked(op);
    if (!out || !fric || !V_init || !theta_init || !tau0) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    if (n_variants != op->h.n_variants)
      throw Error(SEAS_ERR_INVALID_ARG, "n_variants must equal the operator's (" + std::to_string(op->h.n_variants) + ")");
    if (!fric->a || !fric->b || !fric->Dc || !fric->sigma_n || !fric->V0 || !fric->f0)
      throw Error(SEAS_ERR_INVALID_ARG, "null friction array");
    *out = nullptr;
    const HostOp& h = op->h;
    const int nv = n_variants;
    const size_t N = (size_t)h.N * nv;  // values of a per-element array over all variants
    hipStream_t s = (hipStream_t)stream;
    auto st = std::make_unique<seas_state>();
    st->op = op;
    st->nv = nv;
    auto A = [&](size_t bytes, bool ck) {
      void* p = dalloc(st->owned, bytes);
      HIPCHK(hipMemsetAsync(p, 0, bytes, s));
      if (ck) st->ckpt.push_back({p, bytes});
      return p;
    };
    const size_t vb = N * 8;
    st->V = (double*)A(vb, true);
    st->theta = (double*)A(vb, true);
    st->thdot = (double*)A(vb, true);
    st->delta = (double*)A(vb, true);
    st->tau0 = (double*)A(vb, true);
    st->tau0_rate = (double*)A(vb, true);
    st->fa = (double*)A(vb, true);
    st->fb = (double*)A(vb, true);
    st->fDc = (double*)A(vb, true);
    st->fsn = (double*)A(vb, true);
    st->fV0 = (double*)A(vb, true);
    st->ff0 = (double*)A(vb, true);
    st->feps = (double*)A(vb, true);
    st->Vstar = (double*)A(vb, false);
    st->Vbar = (double*)A(vb, false);
    st->th2 = (double*)A(vb, false);
    st->f_hist = (double*)A(vb, true);
    st->f_self = (double*)A(vb, true);
    st->f_int = (double*)A(vb, true);
    st->step0 = (int64_t*)A((size_t)nv * 8, true);
    st->ring64 = (double*)A((size_t)h.ring_len * vb, true);
    st->ringop = op->ring_bytes == 8 ? (void*)st->ring64 : A((size_t)h.ring_len * N * op->ring_bytes, true);
    st->tail_acc = (double*)A((size_t)h.tail_len * 8 * nv, true);
    // item kernels: FP64 slots even where the far pass writes FP32, since the plain
    // form of an FP32 build (seas_state_set_time_block(1)) writes FP64 partials into
    // the same buffer; the segment kernel writes FP32 partials in either form
    st->partials_far = A((size_t)h.n_partials[0] * (h.seg ? 4 : 8), false);
    st->partials_near = (double*)A((size_t)h.n_partials[1] * 8, false);
    st->f_far = (double*)A((size_t)h.time_block * vb, true);
    st->dring = (double2*)A((size_t)h.self_ring_len * 16 * nv, true);
    st->Fh = (double2*)A((size_t)h.n_modes * 16 * nv, false);
    st->F = (double2*)A((size_t)h.n_modes * 16 * nv, false);
    st->fail = (int*)A((size_t)nv * sizeof(int), true);
    st->good = (int64_t*)A((size_t)nv * sizeof(int64_t), true);
    st->V2 = (double*)A(vb, false);
    st->td2 = (double*)A(vb, false);
    st->fs2 = (double*)A(vb, false);
    st->fi2 = (double*)A(vb, false);
    st->Dnew = (double2*)A((size_t)h.n_modes * 16 * nv, false);
    if (h.prm.adaptive_dt) {
      st->dtev = (double*)A(kDtEvBlocks * sizeof(double), false);
      st->Dsv = (double2*)A((size_t)h.n_modes * 16 * nv, false);
    }
    // host-side initial values
    std::vector<double> eps(N, 1.0), thd(N), zero(N, 0.0);
    if (fric->eps) eps.assign(fric->eps, fric->eps + N);
    for (size_t r = 0; r < N; ++r) {
      if (!(V_init[r] > 0) || !(theta_init[r] > 0) || !(fric->Dc[r] > 0) || !(fric->V0[r] > 0) ||
          !(eps[r] > 0 && eps[r] <= 1.0))
        throw Error(SEAS_ERR_INVALID_ARG, "V, theta, Dc, V0 must be > 0 and 0 < eps <= 1");
      thd[r] = host_state_rate(V_init[r], theta_init[r], fric->Dc[r], eps[r]);
    }
    auto H2D = [&](void* d, const double* src) { HIPCHK(hipMemcpyAsync(d, src, vb, hipMemcpyHostToDevice, s)); };
    H2D(st->V, V_init);
    H2D(st->theta, theta_init);
    H2D(st->thdot, thd.data());
    H2D(st->delta, delta_init ? delta_init : zero.data());
    H2D(st->tau0, tau0);
    H2D(st->tau0_rate, tau0_rate ? tau0_rate : zero.data());
    H2D(st->fa, fric->a);
    H2D(st->fb, fric->b);
    H2D(st->fDc, fric->Dc);
    H2D(st->fsn, fric->sigma_n);
    H2D(st->fV0, fric->V0);
    H2D(st->ff0, fric->f0);
    H2D(st->feps, eps.data());
    // histories at t = 0: V^0 and D^0
    H2D(st->ring64, V_init);  // time 0 -> slot 0
    upload_op_row(op, st->ringop, 0, V_init, N, s);
    launch_dft(h.n_modes, nv, h.N, h.self_ring_len, op->modes, op->sf, st->delta, nullptr, 0.0, op->tw, op->tab,
               nullptr, st->F, st->dring, 1, 0, 0, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    *out = st.release();
  });
}

void seas_state_destroy(seas_state_t* st) {
  if (st) {
    (void)hipSetDevice(st->op->device);
    delete st;
  }
}

seas_status seas_state_load_history(seas_state_t* st, const double* V_hist, int32_t n_hist, void* stream) {
  return guard([&] {
    if (!st || (!V_hist && n_hist > 0) || n_hist < 0) throw Error(SEAS_ERR_INVALID_ARG, "bad argument");
    seas_op* op = checked(st->op);
    if (st->mode != 0 || st->step != 0) throw Error(SEAS_ERR_MISMATCH, "history must be loaded on a fresh state");
    if (n_hist == 0) return;
    const HostOp& h = op->h;
    const int nv = st->nv;
    const size_t Ne = h.N, N = Ne * nv;
    hipStream_t s = (hipStream_t)stream;
    const int64_t H = n_hist;
    // rate rows m = -H..-1 (row H + m of V_hist, nv x N values); only the newest
    // ring_len - 2 can be read
    const int64_t mlo = std::max<int64_t>(-H, -(int64_t)(h.ring_len - 2));
    for (int64_t m = mlo; m <= -1; ++m) {
      const double* row = V_hist + (size_t)(H + m) * N;
      const int64_t slot = ((m % h.ring_len) + h.ring_len) % h.ring_len;
      HIPCHK(hipMemcpyAsync(st->ring64 + slot * N, row, N * 8, hipMemcpyHostToDevice, s));
      upload_op_row(op, st->ringop, slot, row, N, s);
    }
    // slip before t = 0 and its coefficients D^m, m = -1 .. 1 - W_max
    std::vector<double> d0(N);
    HIPCHK(hipMemcpyAsync(d0.data(), st->delta, N * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t dlo = std::max<int64_t>(-H, 1 - (int64_t)std::max(1, h.max_self_W));
    double* dtmp = (double*)dalloc(st->owned, N * 8);
    std::vector<double> dm(d0);
    for (int64_t m = -1; m >= dlo; --m) {
      const double* row = V_hist + (size_t)(H + m) * N;
      for (size_t r = 0; r < N; ++r) dm[r] -= h.dt * row[r];
      HIPCHK(hipMemcpyAsync(dtmp, dm.data(), N * 8, hipMemcpyHostToDevice, s));
      launch_dft(h.n_modes, nv, h.N, h.self_ring_len, op->modes, op->sf, dtmp, nullptr, 0.0, op->tw, op->tab,
                 nullptr, st->F, st->dring, 1, m, 0, s);
      HIPCHK(hipStreamSynchronize(s));
    }
    // expired-slip accumulators: dt sum of V^m, m <= -T_end - 1, for every
    // (accumulator, upper lag) entry of every source element
    if (h.prm.int_tail) {
      std::vector<double> E((size_t)h.tail_len * nv, 0.0);
      for (int v = 0; v < nv; ++v)
        for (size_t r = 0; r < Ne; ++r)
          for (int32_t e = h.tail_src_ptr[r]; e < h.tail_src_ptr[r + 1]; ++e) {
            const int32_t acc = h.tail_src[2 * e], Tend = h.tail_src[2 * e + 1];
            double sum = 0.0;
            for (int64_t m = -H; m <= -(int64_t)Tend - 1; ++m) sum += h.dt * V_hist[(size_t)(H + m) * N + (size_t)v * Ne + r];
            E[(size_t)v * h.tail_len + acc] += sum;
          }
      HIPCHK(hipMemcpyAsync(st->tail_acc, E.data(), E.size() * 8, hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    st->first = -H;
  });
}

seas_status seas_state_reset_variant(seas_state_t* st, int32_t variant, const seas_friction_t* fric,
                                     const double* V_init, const double* theta_init, const double* tau0,
                                     const double* tau0_rate, const double* delta_init, void* stream) {
  return guard([&] {
    if (!st || !fric || !V_init || !theta_init || !tau0) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    seas_op* op = checked(st->op);
    if (variant < 0 || variant >= st->nv) throw Error(SEAS_ERR_INVALID_ARG, "variant out of range");
    if (st->mode == 1) throw Error(SEAS_ERR_MISMATCH, "state is in prescribed-history mode");
    if (!fric->a || !fric->b || !fric->Dc || !fric->sigma_n || !fric->V0 || !fric->f0)
      throw Error(SEAS_ERR_INVALID_ARG, "null friction array");
    const HostOp& h = op->h;
    const int nv = st->nv, v = variant;
    const size_t N = h.N;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> eps(N, 1.0), thd(N), zero(N, 0.0);
    if (fric->eps) eps.assign(fric->eps, fric->eps + N);
    for (size_t r = 0; r < N; ++r) {
      if (!(V_init[r] > 0) || !(theta_init[r] > 0) || !(fric->Dc[r] > 0) || !(fric->V0[r] > 0) ||
          !(eps[r] > 0 && eps[r] <= 1.0))
        throw Error(SEAS_ERR_INVALID_ARG, "V, theta, Dc, V0 must be > 0 and 0 < eps <= 1");
      thd[r] = host_state_rate(V_init[r], theta_init[r], fric->Dc[r], eps[r]);
    }
    const size_t o = (size_t)v * N;
    auto H2D = [&](double* d, const double* src) {
      HIPCHK(hipMemcpyAsync(d + o, src, N * 8, hipMemcpyHostToDevice, s));
    };
    H2D(st->V, V_init);
    H2D(st->theta, theta_init);
    H2D(st->thdot, thd.data());
    H2D(st->delta, delta_init ? delta_init : zero.data());
    H2D(st->tau0, tau0);
    H2D(st->tau0_rate, tau0_rate ? tau0_rate : zero.data());
    H2D(st->fa, fric->a);
    H2D(st->fb, fric->b);
    H2D(st->fDc, fric->Dc);
    H2D(st->fsn, fric->sigma_n);
    H2D(st->fV0, fric->V0);
    H2D(st->ff0, fric->f0);
    H2D(st->feps, eps.data());
    const int64_t n = st->step;
    const int zero_flag = 0;
    HIPCHK(hipMemcpyAsync(st->step0 + v, &n, 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(st->good + v, &n, 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(st->fail + v, &zero_flag, sizeof(int), hipMemcpyHostToDevice, s));
    // no history before the variant's start: clear its rows of every ring, then
    // append V^n and the coefficients of its slip at n
    launch_clear_variant(st->ring64, h.ring_len, nv, v, h.N, 8, s);
    if (op->ring_bytes == 2)  // [R][N][nv]
      launch_clear_variant(st->ringop, (int64_t)h.ring_len * h.N, nv, v, 1, 2, s);
    else if (op->ring_bytes != 8)
      launch_clear_variant(st->ringop, h.ring_len, nv, v, h.N, (int)op->ring_bytes, s);
    launch_clear_variant(st->dring, 1, nv, v, (int)(h.self_ring_len * 2), 8, s);
    launch_clear_variant(st->tail_acc, 1, nv, v, (int)h.tail_len, 8, s);
    const int64_t slot = ((n % h.ring_len) + h.ring_len) % h.ring_len;
    HIPCHK(hipMemcpyAsync(st->ring64 + ((size_t)slot * nv + v) * N, V_init, N * 8, hipMemcpyHostToDevice, s));
    if (op->ring_bytes == 2) upload_op_variant(op, st->ringop, slot, nv, v, V_init, s);
    else upload_op_seg(op, st->ringop, ((size_t)slot * nv + v) * N, V_init, N, s);
    launch_dft(h.n_modes, 1, h.N, h.self_ring_len, op->modes, op->sf, st->delta + o, nullptr, 0.0, op->tw, op->tab,
               nullptr, st->F + (size_t)v * h.n_modes, st->dring + (size_t)v * h.self_ring_len, 1, n, n, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));  // the host arrays above are temporaries
    if (st->mode == 0) st->mode = 2;
  });
}

seas_status seas_eval_prescribed(seas_op_t* op, seas_state_t* st, const double* V_dev, int32_t n_steps, double* f_dev,
                                 void* stream) {
  return guard([&] {
    checked(op);
    if (!st || st->op != op) throw Error(SEAS_ERR_MISMATCH, "state belongs to another operator");
    if (n_steps < 0 || (n_steps > 0 && (!V_dev || !f_dev))) throw Error(SEAS_ERR_INVALID_ARG, "bad arguments");
    if (st->mode == 2) throw Error(SEAS_ERR_MISMATCH, "state has taken SEAS steps");
    st->mode = 1;
    hipStream_t s = (hipStream_t)stream;
    switch (op->ring_bytes) {
      case 8: do_prescribed<double>(op, st, V_dev, n_steps, f_dev, s); break;
      case 4: do_prescribed<float>(op, st, V_dev, n_steps, f_dev, s); break;
      default: do_prescribed<__bf16>(op, st, V_dev, n_steps, f_dev, s); break;
    }
  });
}

seas_status seas_eval_prescribed_noalloc(seas_op_t* op, seas_state_t* st, const double* V_dev, int32_t n_steps,
                                         double* f_dev, void* stream) {
  return guard([&] {
    checked(op);  // makes the operator's device current
    if (!st || st->op != op) throw Error(SEAS_ERR_MISMATCH, "state belongs to another operator");
    if (n_steps < 0 || (n_steps > 0 && (!V_dev || !f_dev))) throw Error(SEAS_ERR_INVALID_ARG, "bad arguments");
    if (st->mode == 2) throw Error(SEAS_ERR_MISMATCH, "state has taken SEAS steps");
    const std::pair<size_t, size_t> lay = partial_layout(op->h);
    if (lay.second > kScratchBytes)
      throw Error(SEAS_ERR_INVALID_ARG, "the operator's partial sums need " + std::to_string(lay.second) +
                                            " bytes; the static scratch holds " + std::to_string(kScratchBytes));
    if (st->timing) throw Error(SEAS_ERR_MISMATCH, "kernel timing (which creates events) is on for this state");
    unsigned char* base = (unsigned char*)scratch_ptr(op->device);
    st->mode = 1;
    hipStream_t s = (hipStream_t)stream;
    void* pfar = base;
    double* pnear = (double*)(base + lay.first);
    switch (op->ring_bytes) {
      case 8: do_prescribed<double>(op, st, V_dev, n_steps, f_dev, s, pfar, pnear); break;
      case 4: do_prescribed<float>(op, st, V_dev, n_steps, f_dev, s, pfar, pnear); break;
      default: do_prescribed<__bf16>(op, st, V_dev, n_steps, f_dev, s, pfar, pnear); break;
    }
  });
}

seas_status seas_step(seas_op_t* op, seas_state_t* st, int32_t n_steps, void* stream) {
  return guard([&] {
    checked(op);
    if (!st || st->op != op) throw Error(SEAS_ERR_MISMATCH, "state belongs to another operator");
    if (n_steps < 0) throw Error(SEAS_ERR_INVALID_ARG, "n_steps < 0");
    if (st->mode == 1) throw Error(SEAS_ERR_MISMATCH, "state is in prescribed-history mode");
    st->mode = 2;
    hipStream_t s = (hipStream_t)stream;
    switch (op->ring_bytes) {
      case 8: do_steps<double>(op, st, n_steps, s); break;
      case 4: do_steps<float>(op, st, n_steps, s); break;
      default: do_steps<__bf16>(op, st, n_steps, s); break;
    }
  });
}

seas_status seas_state_check(seas_state_t* st, void* stream) {
  std::vector<int> bad;
  std::vector<int64_t> good;
  seas_status rc = guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    checked(st->op);
    hipStream_t s = (hipStream_t)stream;
    bad.assign(st->nv, 0);
    good.assign(st->nv, 0);
    HIPCHK(hipMemcpyAsync(bad.data(), st->fail, st->nv * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(good.data(), st->good, st->nv * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st->nv == 1 && bad[0]) {
      // one variant: the state is back at its last good step, ready to resume
      st->step = good[0];
      st->block_head = INT64_MIN / 2;
      HIPCHK(hipMemsetAsync(st->fail, 0, sizeof(int), s));
      HIPCHK(hipStreamSynchronize(s));
    }
  });
  if (rc != SEAS_OK) return rc;
  std::string msg;
  for (size_t v = 0; v < bad.size(); ++v)
    if (bad[v]) {
      if (msg.empty()) msg = "Newton did not converge within 50 iterations: ";
      else msg += ", ";
      msg += "variant " + std::to_string(v) + " held at step " + std::to_string(good[v]);
    }
  if (!msg.empty()) {
    g_err = msg;
    return SEAS_ERR_NOT_CONVERGED;
  }
  return SEAS_OK;
}

seas_status seas_state_variant_status(const seas_state_t* st, int32_t* failed, int64_t* good_step, void* stream) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    checked(st->op);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> bad(st->nv);
    if (failed) {
      HIPCHK(hipMemcpyAsync(bad.data(), st->fail, st->nv * sizeof(int), hipMemcpyDeviceToHost, s));
    }
    if (good_step) HIPCHK(hipMemcpyAsync(good_step, st->good, st->nv * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (failed)
      for (int v = 0; v < st->nv; ++v) failed[v] = bad[v];
  });
}

seas_status seas_write_state(seas_state_t* st, int32_t field, int32_t variant, const double* src, size_t count,
                             int32_t src_is_device, void* stream) {
  return guard([&] {
    if (!st || !src) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    seas_op* op = checked(st->op);
    if (variant < 0 || variant >= st->nv) throw Error(SEAS_ERR_INVALID_ARG, "variant out of range");
    const HostOp& h = op->h;
    const size_t N = h.N;
    if (count != N) throw Error(SEAS_ERR_INVALID_ARG, "count must equal the number of elements");
    if (st->mode == 1) throw Error(SEAS_ERR_MISMATCH, "state is in prescribed-history mode");
    hipStream_t s = (hipStream_t)stream;
    const int nv = st->nv, v = variant;
    const size_t o = (size_t)v * N;
    std::vector<double> x(src_is_device ? N : 0);
    const double* hx = src;
    if (src_is_device) {
      HIPCHK(hipMemcpyAsync(x.data(), src, N * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      hx = x.data();
    }
    double* dst = nullptr;
    switch (field) {
      case SEAS_FIELD_V:
        for (size_t r = 0; r < N; ++r)
          if (!(hx[r] > 0)) throw Error(SEAS_ERR_INVALID_ARG, "V must be > 0");
        dst = st->V;
        break;
      case SEAS_FIELD_THETA:
        for (size_t r = 0; r < N; ++r)
          if (!(hx[r] > 0)) throw Error(SEAS_ERR_INVALID_ARG, "theta must be > 0");
        dst = st->theta;
        break;
      case SEAS_FIELD_DELTA: dst = st->delta; break;
      case SEAS_FIELD_TAU0: dst = st->tau0; break;
      default: throw Error(SEAS_ERR_INVALID_ARG, "field cannot be written (V, THETA, DELTA or TAU0)");
    }
    HIPCHK(hipMemcpyAsync(dst + o, hx, N * 8, hipMemcpyHostToDevice, s));
    const int64_t n = st->step;
    if (field == SEAS_FIELD_V) {
      // V^n is also the newest row of the rate history
      const int64_t slot = ((n % h.ring_len) + h.ring_len) % h.ring_len;
      HIPCHK(hipMemcpyAsync(st->ring64 + ((size_t)slot * nv + v) * N, hx, N * 8, hipMemcpyHostToDevice, s));
      if (op->ring_bytes == 2) upload_op_variant(op, st->ringop, slot, nv, v, hx, s);
      else upload_op_seg(op, st->ringop, ((size_t)slot * nv + v) * N, hx, N, s);
    }
    if (field == SEAS_FIELD_V || field == SEAS_FIELD_THETA) {
      // the state rate follows from V and theta
      std::vector<double> V(N), th(N), Dc(N), eps(N), thd(N);
      HIPCHK(hipMemcpyAsync(V.data(), st->V + o, N * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(th.data(), st->theta + o, N * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(Dc.data(), st->fDc + o, N * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(eps.data(), st->feps + o, N * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (size_t r = 0; r < N; ++r) thd[r] = host_state_rate(V[r], th[r], Dc[r], eps[r]);
      HIPCHK(hipMemcpyAsync(st->thdot + o, thd.data(), N * 8, hipMemcpyHostToDevice, s));
    }
    if (field == SEAS_FIELD_DELTA) {
      // D^n, the transform of the slip at the current step, is the newest coefficient row
      launch_dft(h.n_modes, 1, h.N, h.self_ring_len, op->modes, op->sf, st->delta + o, nullptr, 0.0, op->tw,
                 op->tab, nullptr, st->F + (size_t)v * h.n_modes, st->dring + (size_t)v * h.self_ring_len, 1, n, n, s);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    if (st->mode == 0) st->mode = 2;
  });
}

seas_status seas_read_state(const seas_state_t* st, int32_t field, int32_t variant, double* dst, size_t count,
                            int32_t dst_is_device, void* stream) {
  return guard([&] {
    if (!st || !dst) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    checked(st->op);
    if (variant < 0 || variant >= st->nv) throw Error(SEAS_ERR_INVALID_ARG, "variant out of range");
    const size_t N = st->op->h.N;
    if (count != N) throw Error(SEAS_ERR_INVALID_ARG, "count must equal the number of elements");
    const double* src = nullptr;
    switch (field) {
      case SEAS_FIELD_V: src = st->V; break;
      case SEAS_FIELD_THETA: src = st->theta; break;
      case SEAS_FIELD_DELTA: src = st->delta; break;
      case SEAS_FIELD_THETADOT: src = st->thdot; break;
      case SEAS_FIELD_F_HIST: src = st->f_hist; break;
      case SEAS_FIELD_F_SELF: src = st->f_self; break;
      case SEAS_FIELD_F_INT: src = st->f_int; break;
      case SEAS_FIELD_TAU0: src = st->tau0; break;
      default: throw Error(SEAS_ERR_INVALID_ARG, "unknown field");
    }
    src += (size_t)variant * N;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(dst, src, N * 8, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dst_is_device) HIPCHK(hipStreamSynchronize(s));
  });
}

int64_t seas_state_step_index(const seas_state_t* st) { return st ? st->step : -1; }

seas_status seas_state_set_timing(seas_state_t* st, int32_t enable) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    st->timing = enable != 0;
  });
}

seas_status seas_state_set_gamma_cap(seas_state_t* st, int64_t cap) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    if (cap < 0) throw Error(SEAS_ERR_INVALID_ARG, "cap < 0");
    st->gamma_cap = cap;
  });
}

seas_status seas_state_progress(const seas_state_t* st, int64_t* steps_taken, int64_t* last_gamma, double* time_s) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    if (steps_taken) *steps_taken = st->steps_taken;
    if (last_gamma) *last_gamma = st->last_gamma;
    if (time_s) *time_s = (double)st->step * st->op->h.dt;
  });
}

seas_status seas_operator_set_tune(seas_op_t* op, int32_t variant) {
  return guard([&] {
    checked(op);
    if (variant < 0 || variant >= kTuneVariants) throw Error(SEAS_ERR_INVALID_ARG, "no such variant");
    op->h.x16_tune = variant;
  });
}

seas_status seas_operator_tune(seas_op_t* op, seas_state_t* st, void* stream, int32_t reps, double* ms,
                               int32_t* choice) {
  return guard([&] {
    checked(op);
    if (!st || st->op != op) throw Error(SEAS_ERR_MISMATCH, "state belongs to another operator");
    if (reps < 1) throw Error(SEAS_ERR_INVALID_ARG, "reps >= 1");
    HostOp& h = op->h;
    const bool tunable = h.seg;
    if (ms)
      for (int c = 0; c < kTuneVariants; ++c) ms[c] = -1.0;
    if (!tunable) {
      if (choice) *choice = h.x16_tune;
      return;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int S = h.time_block;
    const int64_t head = st->step;
    int best = 0;
    double best_ms = 0.0;
    try {
      for (int c = 0; c < kTuneVariants; ++c) {
        h.x16_tune = c;
        // the far sums of a whole time block land in the state's partial buffer,
        // which the next block start overwrites before reading (ensembles: every step)
        const FarPart part = S > 1 ? kFarRest : kFarAll;
        launch_far(op, st, head, part, S, st->partials_far, s);
        HIPCHK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch_far(op, st, head, part, S, st->partials_far, s);
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        const double per = (double)t / reps;
        if (ms) ms[c] = per;
        if (c == 0 || per < best_ms) {
          best = c;
          best_ms = per;
        }
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      h.x16_tune = 0;
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h.x16_tune = best;
    if (choice) *choice = best;
  });
}

seas_status seas_state_set_graph(seas_state_t* st, int32_t enable) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    checked(st->op);
    if (enable && st->op->h.prm.adaptive_dt)
      throw Error(SEAS_ERR_MISMATCH, "adaptive steps choose each step's length on the host");
    if (enable && !st->clk) st->clk = (int64_t*)dalloc(st->owned, 256);
    st->graph = enable != 0;
  });
}

seas_status seas_state_graph_info(const seas_state_t* st, int64_t* replays, int32_t* steps_per_replay) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    if (replays) *replays = st->g_replays;
    if (steps_per_replay) *steps_per_replay = st->gexec ? st->g_unit : 0;
  });
}

seas_status seas_state_set_overlap(seas_state_t* st, int32_t enable) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    st->overlap = enable != 0;
  });
}

seas_status seas_state_set_time_block(seas_state_t* st, int32_t S) {
  return guard([&] {
    if (!st) throw Error(SEAS_ERR_INVALID_ARG, "null state");
    if (S != 1 && S != st->op->h.time_block) throw Error(SEAS_ERR_INVALID_ARG, "S must be 1 or the build's time_block");
    st->run_S = S;
    st->block_head = INT64_MIN / 2;
  });
}

seas_status seas_state_read_timing(seas_state_t* st, void* stream, double* ms_total, int64_t* launches) {
  return guard([&] {
    if (!st || !ms_total || !launches) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    checked(st->op);
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    double tot = 0.0;
    for (size_t i = 0; i < st->n_ev; ++i) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, st->ev[2 * i], st->ev[2 * i + 1]));
      tot += ms;
    }
    *ms_total = tot;
    *launches = (int64_t)st->n_ev;
    st->n_ev = 0;
  });
}

size_t seas_state_checkpoint_bytes(const seas_state_t* st) {
  if (!st) return 0;
  size_t b = 5 * sizeof(int64_t);
  for (auto& c : st->ckpt) b += c.bytes;
  return b;
}

seas_status seas_state_save(const seas_state_t* st, void* host_buf, size_t bytes, void* stream) {
  return guard([&] {
    if (!st || !host_buf) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    checked(st->op);
    if (bytes < seas_state_checkpoint_bytes(st)) throw Error(SEAS_ERR_INVALID_ARG, "buffer too small");
    hipStream_t s = (hipStream_t)stream;
    char* p = (char*)host_buf;
    const int64_t hdr[5] = {st->step, st->first, st->mode, (int64_t)st->op->h.N, st->block_head};
    std::memcpy(p, hdr, sizeof(hdr));
    p += sizeof(hdr);
    for (auto& c : st->ckpt) {
      HIPCHK(hipMemcpyAsync(p, c.p, c.bytes, hipMemcpyDeviceToHost, s));
      p += c.bytes;
    }
    HIPCHK(hipStreamSynchronize(s));
  });
}

seas_status seas_state_restore(seas_state_t* st, const void* host_buf, size_t bytes, void* stream) {
  return guard([&] {
    if (!st || !host_buf) throw Error(SEAS_ERR_INVALID_ARG, "null argument");
    checked(st->op);
    if (bytes < seas_state_checkpoint_bytes(st)) throw Error(SEAS_ERR_INVALID_ARG, "buffer too small");
    const char* p = (const char*)host_buf;
    int64_t hdr[5];
    std::memcpy(hdr, p, sizeof(hdr));
    if (hdr[3] != st->op->h.N) throw Error(SEAS_ERR_MISMATCH, "checkpoint of another operator");
    p += sizeof(hdr);
    hipStream_t s = (hipStream_t)stream;
    for (auto& c : st->ckpt) {
      HIPCHK(hipMemcpyAsync(c.p, p, c.bytes, hipMemcpyHostToDevice, s));
      p += c.bytes;
    }
    HIPCHK(hipStreamSynchronize(s));
    st->step = hdr[0];
    st->first = hdr[1];
    st->mode = (int)hdr[2];
    st->block_head = hdr[4];
  });
}

}  // extern "C"
