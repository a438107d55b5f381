// Request loop for simulation windows (continuous batching), built on the public
// C ABI of this library.
//
// Every geometry ("pool") owns one ensemble state whose variant slots hold the
// requests of that geometry; the state is created when the first request of
// the pool arrives and the device budget allows its bytes (seas_state_bytes).
// A pool steps its state in chunks of at most `chunk` steps on its own stream,
// so pools overlap on the device. Between chunks, finished requests leave their
// slots (the final state is copied out and the slot returns to the idle window
// given at creation) and waiting requests of the pool take free slots
// (seas_state_reset_variant), so requests join and leave a running batch. A
// chunk never runs past the end of the shortest active window, so every
// request stops exactly after its n_steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

using namespace seas;

namespace {

struct Slot {
  int req = -1;       // request index, -1 when idle
  int64_t done = 0;   // steps taken in this window
};

struct Pool {
  seas_op_t* op = nullptr;
  int nv = 1, N = 0;
  size_t bytes = 0;
  seas_request_t idle{};
  seas_state_t* st = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  int K = 0;  // steps of the chunk in flight
  int64_t stepped = 0;  // steps the pool's state has taken (progress reports)
  std::vector<Slot> slots;
  std::deque<int> waiting;
};

seas_status raise_status(seas_status rc, const char* what) {
  if (rc != SEAS_OK) throw Error(rc, std::string(what) + ": " + seas_last_error());
  return rc;
}

}  // namespace

struct seas_server {
  std::vector<Pool> pools;
  size_t budget = 0, used = 0;
  int chunk = 16;
  ~seas_server() {
    for (auto& p : pools) {
      if (p.st) seas_state_destroy(p.st);
      if (p.ev) (void)hipEventDestroy(p.ev);
      if (p.stream) (void)hipStreamDestroy(p.stream);
    }
  }
};

namespace {

template <typename F>
seas_status sguard(F&& f) {
  try {
    f();
    return SEAS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return SEAS_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SEAS_ERR_INTERNAL;
  }
}

void reset_slot(Pool& p, int slot, const seas_request_t& r) {
  raise_status(seas_state_reset_variant(p.st, slot, &r.fric, r.V_init, r.theta_init, r.tau0, r.tau0_rate,
                                        r.delta_init, p.stream),
               "seas_state_reset_variant");
}

void create_state(Pool& p) {
  const size_t n = (size_t)p.N * p.nv;
  const seas_request_t& r = p.idle;
  auto tile = [&](const double* src, std::vector<double>& dst) {
    dst.resize(n);
    for (int v = 0; v < p.nv; ++v) std::copy(src, src + p.N, dst.begin() + (size_t)v * p.N);
  };
  std::vector<double> a, b, Dc, sn, V0, f0, eps, V, th, t0, t0r, d0;
  tile(r.fric.a, a);
  tile(r.fric.b, b);
  tile(r.fric.Dc, Dc);
  tile(r.fric.sigma_n, sn);
  tile(r.fric.V0, V0);
  tile(r.fric.f0, f0);
  tile(r.V_init, V);
  tile(r.theta_init, th);
  tile(r.tau0, t0);
  if (r.fric.eps) tile(r.fric.eps, eps);
  if (r.tau0_rate) tile(r.tau0_rate, t0r);
  if (r.delta_init) tile(r.delta_init, d0);
  seas_friction_t fr{a.data(), b.data(), Dc.data(), sn.data(), V0.data(), f0.data(),
                     r.fric.eps ? eps.data() : nullptr};
  raise_status(seas_state_create(p.op, p.nv, &fr, V.data(), th.data(), t0.data(),
                                 r.tau0_rate ? t0r.data() : nullptr, r.delta_init ? d0.data() : nullptr, p.stream,
                                 &p.st),
               "seas_state_create");
  p.slots.assign(p.nv, Slot{});
}

}  // namespace

extern "C" {

seas_status seas_server_create(seas_op_t* const* ops, int32_t n_ops, const seas_request_t* idle,
                               size_t device_budget, int32_t chunk_steps, seas_server_t** out) {
  return sguard([&] {
    if (!ops || !idle || !out || n_ops < 1 || chunk_steps < 1) throw Error(SEAS_ERR_INVALID_ARG, "bad argument");
    *out = nullptr;
    auto sv = std::make_unique<seas_server>();
    sv->budget = device_budget;
    sv->chunk = chunk_steps;
    sv->pools.resize(n_ops);
    for (int k = 0; k < n_ops; ++k) {
      Pool& p = sv->pools[k];
      if (!ops[k]) throw Error(SEAS_ERR_INVALID_ARG, "null operator");
      seas_op_info_t info;
      raise_status(seas_operator_info(ops[k], &info), "seas_operator_info");
      p.op = ops[k];
      p.nv = info.n_variants;
      p.N = info.n_elem;
      p.bytes = seas_state_bytes(ops[k], p.nv);
      p.idle = idle[k];
      if (!p.idle.V_init || !p.idle.theta_init || !p.idle.tau0 || !p.idle.fric.a || !p.idle.fric.b ||
          !p.idle.fric.Dc || !p.idle.fric.sigma_n || !p.idle.fric.V0 || !p.idle.fric.f0)
        throw Error(SEAS_ERR_INVALID_ARG, "idle window of pool " + std::to_string(k) + " incomplete");
      if (p.bytes > device_budget)
        throw Error(SEAS_ERR_INVALID_ARG, "pool " + std::to_string(k) + " needs more than the device budget");
      if (hipStreamCreate(&p.stream) != hipSuccess || hipEventCreateWithFlags(&p.ev, hipEventDisableTiming) !=
                                                          hipSuccess)
        throw Error(SEAS_ERR_HIP, "stream or event creation failed");
    }
    *out = sv.release();
  });
}

seas_status seas_server_run(seas_server_t* sv, seas_request_t* rq, int32_t n) {
  return sguard([&] {
    if (!sv || (!rq && n > 0) || n < 0) throw Error(SEAS_ERR_INVALID_ARG, "bad argument");
    for (int i = 0; i < n; ++i) {
      if (rq[i].pool < 0 || rq[i].pool >= (int)sv->pools.size() || rq[i].n_steps < 1)
        throw Error(SEAS_ERR_INVALID_ARG, "request " + std::to_string(i) + ": bad pool or n_steps");
      rq[i].admit_s = rq[i].finish_s = -1.0;
      rq[i].status = SEAS_OK;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rq[x].arrival_s < rq[y].arrival_s; });
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    // SEAS_VERBOSE: a line on stderr per finished request and per 1000 steps of a pool
    const bool verbose = std::getenv("SEAS_VERBOSE") != nullptr;
    int next = 0, finished = 0;
    while (finished < n) {
      bool progress = false;
      const double t = now();
      while (next < n && rq[order[next]].arrival_s <= t) {
        sv->pools[rq[order[next]].pool].waiting.push_back(order[next]);
        ++next;
      }
      for (Pool& p : sv->pools) {
        // completions of the chunk in flight
        if (p.busy) {
          const hipError_t q = hipEventQuery(p.ev);
          if (q == hipErrorNotReady) continue;
          if (q != hipSuccess) throw Error(SEAS_ERR_HIP, "hipEventQuery failed");
          p.busy = false;
          progress = true;
          if (verbose && (p.stepped + p.K) / 1000 != p.stepped / 1000)
            std::fprintf(stderr, "[seas server] %.1f s: pool %d at step %lld\n", now(), (int)(&p - &sv->pools[0]),
                         (long long)(p.stepped + p.K));
          p.stepped += p.K;
          // a slot whose Newton solve failed is held at its last good step; the
          // others are not affected
          std::vector<int32_t> failed(p.nv, 0);
          raise_status(seas_state_variant_status(p.st, failed.data(), nullptr, p.stream),
                       "seas_state_variant_status");
          for (int s = 0; s < p.nv; ++s) {
            Slot& sl = p.slots[s];
            if (sl.req < 0) {
              if (failed[s]) reset_slot(p, s, p.idle);
              continue;
            }
            sl.done += p.K;
            seas_request_t& r = rq[sl.req];
            if (failed[s]) r.status = SEAS_ERR_NOT_CONVERGED;
            if (sl.done < r.n_steps && !failed[s]) continue;
            double* outs[3] = {r.V_out, r.theta_out, r.delta_out};
            const int32_t fields[3] = {SEAS_FIELD_V, SEAS_FIELD_THETA, SEAS_FIELD_DELTA};
            for (int k = 0; k < 3; ++k)
              if (outs[k])
                raise_status(seas_read_state(p.st, fields[k], s, outs[k], (size_t)p.N, 0, p.stream), "seas_read_state");
            r.finish_s = now();
            ++finished;
            if (verbose)
              std::fprintf(stderr, "[seas server] %.1f s: request %d done (%d of %d)\n", r.finish_s, sl.req, finished,
                           n);
            sl = Slot{};
            reset_slot(p, s, p.idle);  // the slot idles until the next request takes it
          }
        }
        // admission: a state for the pool, then free slots for waiting requests
        if (!p.waiting.empty() && !p.st && sv->used + p.bytes <= sv->budget) {
          create_state(p);
          sv->used += p.bytes;
        }
        if (p.st && !p.busy) {
          for (int s = 0; s < p.nv && !p.waiting.empty(); ++s) {
            if (p.slots[s].req >= 0) continue;
            const int i = p.waiting.front();
            p.waiting.pop_front();
            reset_slot(p, s, rq[i]);
            p.slots[s].req = i;
            p.slots[s].done = 0;
            rq[i].admit_s = now();
            progress = true;
          }
          // next chunk: up to the end of the shortest active window
          int64_t K = sv->chunk;
          bool any = false;
          for (const Slot& sl : p.slots)
            if (sl.req >= 0) {
              any = true;
              K = std::min<int64_t>(K, rq[sl.req].n_steps - sl.done);
            }
          if (any) {
            p.K = (int)K;
            raise_status(seas_step(p.op, p.st, p.K, p.stream), "seas_step");
            if (hipEventRecord(p.ev, p.stream) != hipSuccess) throw Error(SEAS_ERR_HIP, "hipEventRecord failed");
            p.busy = true;
            progress = true;
          } else if (p.waiting.empty()) {
            // idle: give the memory back when another pool waits for it, or when no
            // later request of this pool is in the trace
            const int me = (int)(&p - &sv->pools[0]);
            bool later = false, starved = false;
            for (int j = next; j < n && !later; ++j) later = rq[order[j]].pool == me;
            for (const Pool& o : sv->pools) starved |= !o.waiting.empty() && !o.st;
            if (!later || starved) {
              seas_state_destroy(p.st);
              p.st = nullptr;
              sv->used -= p.bytes;
              progress = true;
            }
          }
        }
      }
      if (!progress) {
        bool busy = false, held = false;
        for (const Pool& p : sv->pools) {
          busy |= p.busy;
          held |= p.st != nullptr;
        }
        if (!busy && next >= n && !held && finished < n)
          throw Error(SEAS_ERR_INTERNAL, "requests left that no pool can admit");
        if (!busy && next < n) {
          const double wait = rq[order[next]].arrival_s - now();
          if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
        } else {
          std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
      }
    }
  });
}

void seas_server_destroy(seas_server_t* sv) { delete sv; }

}  // extern "C"
