// batch.hip - many independent packings stepped together.
//
// Each packing is an ordinary context (its own parameters, domains, walls,
// contact list, tree and order), so a packing's results are those of its
// own cd_step.  Per time step the batch runs every packing's preparation
// (detection, partition, order), then ONE launch per sweep over the domains
// of all packings (each packing's workgroups plus its decision workgroup);
// a packing whose solve has stopped leaves its workgroups idle, and the
// launches end once every packing has stopped.  Then every packing's update.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <thread>
#include <vector>

#include "cd_internal.h"

struct cd_batch {
  std::vector<cd_ctx*> ctx;
  hipStream_t stream = nullptr;
  int dim = 2;
  int grid_total = 0;           // workgroups of one batched sweep launch
  bool staged = false;          // the last batched solve staged contact data in LDS
  SweepArgs* h_tab = nullptr;   // pinned
  SweepArgs* d_tab = nullptr;
  int* d_blk = nullptr;         // per workgroup: packing, workgroup within the packing
  std::vector<int> blk_all;     // the same for every packing (host)
  int* h_blk[2] = {nullptr, nullptr};  // pinned staging of compacted tables
  SolveState* h_states = nullptr;  // pinned
  SolveState* d_states = nullptr;
  BatchProg* h_prog = nullptr;  // mapped pinned
  BatchProg* d_prog = nullptr;
  int time_every = 8;
  std::vector<int> failed;      // per packing: 0, or the error that took it out
  std::vector<hipEvent_t> sweep_ev;
  hipEvent_t ev[4] = {};
  // lanes: the per-packing preparation and update are spread over up to
  // 16 streams, each fed by its own host thread, so that the many small
  // kernels of different packings run side by side
  std::vector<hipStream_t> lane;
  std::vector<hipEvent_t> lane_ev;
  cd_batch_timing timing{};
  std::string err;
};

namespace {

int bfail(cd_batch* b, int code, const std::string& msg) {
  b->err = msg;
  return code;
}

// Host threads (and streams) of the preparation: submission of the many
// small launches scales up to about 16 (measured on 512 packings: 194 ms per
// warm step with one, 100 with four, 78 with eight, 66 with sixteen).
constexpr int kLanes = 16;

// The packings' work on the lanes: packing p on lane p % lanes.
void lanes_attach(cd_batch* b) {
  for (size_t p = 0; p < b->ctx.size(); ++p) b->ctx[p]->stream = b->lane[p % b->lane.size()];
}
void lanes_detach(cd_batch* b) {
  for (cd_ctx* c : b->ctx) c->stream = b->stream;
}

// Every lane waits for what the batch stream has queued so far.
hipError_t lanes_after_batch_stream(cd_batch* b) {
  hipError_t e = hipEventRecord(b->lane_ev[0], b->stream);
  for (size_t t = 0; e == hipSuccess && t < b->lane.size(); ++t)
    e = hipStreamWaitEvent(b->lane[t], b->lane_ev[0], 0);
  return e;
}

// The batch stream waits for everything queued on the lanes.
hipError_t batch_stream_after_lanes(cd_batch* b) {
  hipError_t e = hipSuccess;
  for (size_t t = 0; e == hipSuccess && t < b->lane.size(); ++t) {
    e = hipEventRecord(b->lane_ev[1 + t], b->lane[t]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->lane_ev[1 + t], 0);
  }
  return e;
}

hipError_t lanes_sync(cd_batch* b) {
  hipError_t e = hipSuccess;
  for (hipStream_t s : b->lane)
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// fn(p) for every packing still in the batch, lane t's packings on host
// thread t.  With `soft`, a packing whose step fails with a per-packing
// error (bad input, non-finite state) leaves the batch; any other error is
// returned for the first packing that raised it.
template <class F>
int over_lanes(cd_batch* b, bool soft, F fn) {
  const int B = (int)b->ctx.size(), S = (int)b->lane.size();
  std::vector<int> st(S, CD_OK), at(S, -1);
  auto work = [&](int t) {
    for (int p = t; p < B; p += S) {
      if (b->failed[p]) continue;
      const int r = fn(p);
      if (soft && (r == CD_EINVAL || r == CD_ENONFINITE)) {
        b->failed[p] = r;
        continue;
      }
      if (r != CD_OK) {
        st[t] = r;
        at[t] = p;
        return;
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < S; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  for (int t = 0; t < S; ++t)
    if (st[t] != CD_OK)
      return bfail(b, st[t], "packing " + std::to_string(at[t]) + ": " + cd_last_error(b->ctx[at[t]]));
  return CD_OK;
}

#define BTRY(expr)                                                               \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) return bfail(b, CD_EHIP, hipGetErrorString(e_));       \
  } while (0)

float ms_between(hipEvent_t a, hipEvent_t c) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, c) != hipSuccess) return 0.f;
  return ms;
}

}  // namespace

extern "C" {

int cd_batch_create(cd_batch** out, cd_ctx* const* ctxs, int count) {
  if (!out || !ctxs || count < 1) return CD_EINVAL;
  *out = nullptr;
  cd_batch* b = new cd_batch();
  b->ctx.assign(ctxs, ctxs + count);
  b->stream = ctxs[0]->stream;
  b->dim = ctxs[0]->dim;
  std::vector<int> blk;
  for (int p = 0; p < count; ++p) {
    cd_ctx* c = ctxs[p];
    // walls of finite mass need their own sweep instantiation, which the
    // batched launch does not have
    if (!c || c->stream != b->stream || c->dim != b->dim || c->device != ctxs[0]->device ||
        c->mobile_mask) {
      delete b;
      return CD_EINVAL;
    }
    // the packing's domain workgroups and its decision workgroup
    const int grid = cd_sweep_args(c).grid;
    for (int q = 0; q <= grid; ++q) {
      blk.push_back(p);
      blk.push_back(q);
    }
  }
  b->grid_total = (int)blk.size() / 2;
  b->blk_all = blk;
  b->failed.assign(count, 0);
  int st = CD_OK;
  if (hipHostMalloc((void**)&b->h_tab, sizeof(SweepArgs) * count) != hipSuccess ||
      hipMalloc((void**)&b->d_tab, sizeof(SweepArgs) * count) != hipSuccess ||
      hipHostMalloc((void**)&b->h_states, sizeof(SolveState) * count) != hipSuccess ||
      hipMalloc((void**)&b->d_states, sizeof(SolveState) * count) != hipSuccess ||
      hipMalloc((void**)&b->d_blk, sizeof(int) * blk.size()) != hipSuccess ||
      hipHostMalloc((void**)&b->h_blk[0], sizeof(int) * blk.size()) != hipSuccess ||
      hipHostMalloc((void**)&b->h_blk[1], sizeof(int) * blk.size()) != hipSuccess ||
      hipHostMalloc((void**)&b->h_prog, sizeof(BatchProg), hipHostMallocMapped) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipHostGetDevicePointer((void**)&b->d_prog, b->h_prog, 0) != hipSuccess)
    st = CD_EHIP;
  if (st == CD_OK &&
      hipMemcpy(b->d_blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice) != hipSuccess)
    st = CD_EHIP;
  for (int k = 0; k < 4 && st == CD_OK; ++k)
    if (hipEventCreate(&b->ev[k]) != hipSuccess) st = CD_EHIP;
  const int hw = std::max(1u, std::thread::hardware_concurrency());
  const int lanes = std::min({kLanes, (int)count, (int)hw});
  for (int t = 0; t < lanes && st == CD_OK; ++t) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = CD_EHIP;
    else b->lane.push_back(s);
  }
  for (int t = 0; t <= lanes && st == CD_OK; ++t) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) st = CD_EHIP;
    else b->lane_ev.push_back(e);
  }
  if (st != CD_OK) {
    cd_batch_destroy(b);
    return st;
  }
  // the batch times its own phases: the packings record no events of their
  // own (six per packing and step, a tenth of their host submissions)
  for (cd_ctx* c : b->ctx) c->phase_events = false;
  *out = b;
  return CD_OK;
}

int cd_batch_destroy(cd_batch* b) {
  if (!b) return CD_OK;
  for (cd_ctx* c : b->ctx)
    if (c) c->phase_events = true;
  if (b->h_tab) (void)hipHostFree(b->h_tab);
  if (b->d_tab) (void)hipFree(b->d_tab);
  if (b->h_states) (void)hipHostFree(b->h_states);
  if (b->d_states) (void)hipFree(b->d_states);
  if (b->d_blk) (void)hipFree(b->d_blk);
  for (int k = 0; k < 2; ++k)
    if (b->h_blk[k]) (void)hipHostFree(b->h_blk[k]);
  if (b->h_prog) (void)hipHostFree(b->h_prog);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : b->sweep_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : b->lane_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& s : b->lane)
    if (s) (void)hipStreamDestroy(s);
  delete b;
  return CD_OK;
}

int cd_batch_set_timing(cd_batch* b, int every) {
  if (!b || every < 0) return CD_EINVAL;
  b->time_every = every;
  return CD_OK;
}

int cd_batch_step(cd_batch* b, cd_result* results) {
  if (!b || !results) return CD_EINVAL;
  const int B = (int)b->ctx.size();
  BTRY(hipEventRecord(b->ev[0], b->stream));
  // ---- every packing's preparation, phase by phase with one stream
  // synchronisation between phases for the whole batch.  A packing whose
  // velocities broke the displacement bound or turned non-finite (its solve
  // diverged, Sec. 2.3) leaves the batch: its result carries the error in
  // every later step.
  BTRY(lanes_after_batch_stream(b));
  lanes_attach(b);
  for (int k = 0; k < kPrepPhases; ++k) {
    if (k > 0) {
      hipError_t e = lanes_sync(b);
      if (e != hipSuccess) {
        lanes_detach(b);
        return bfail(b, CD_EHIP, hipGetErrorString(e));
      }
    }
    int st = over_lanes(b, true, [&](int p) { return prep_phase(b->ctx[p], k); });
    if (st != CD_OK) {
      (void)lanes_sync(b);
      lanes_detach(b);
      return st;
    }
  }
  {
    hipError_t e = batch_stream_after_lanes(b);
    lanes_detach(b);
    if (e != hipSuccess) return bfail(b, CD_EHIP, hipGetErrorString(e));
  }
  BTRY(hipEventRecord(b->ev[1], b->stream));
  // ---- the batched solve
  int limit = 0, open = 0, block = 64;
  size_t lds = 8, lds_stage = 8;
  for (int p = 0; p < B; ++p) {
    cd_ctx* c = b->ctx[p];
    if (!b->failed[p] && c->sweep_global)
      return bfail(b, CD_ECAPACITY,
                   "packing " + std::to_string(p) + ": a domain does not fit in LDS");
    if (!b->failed[p] && c->order_mixed)
      return bfail(b, CD_EINVAL,
                   "packing " + std::to_string(p) + ": batched sweeps have no mixed update");
    if (!b->failed[p] && c->order_random)
      return bfail(b, CD_EINVAL,
                   "packing " + std::to_string(p) + ": batched sweeps have no random order");
    b->h_tab[p] = cd_sweep_args(c);
    b->h_tab[p].dtick = nullptr;   // batched sweeps do not measure the load
    block = std::max(block, c->sweep_block);
    lds = std::max(lds, c->sweep_lds);
    lds_stage = std::max(lds_stage, cd_stage_lds(c->st_ds.max_stage +
                                                  (c->use_mu_slot ? 8 * c->st_ds.max_contacts : 0)));
    if (!b->failed[p] && c->nc > 0 && c->st_limit > 0) {
      ++open;
      limit = std::max(limit, c->st_limit);
    }
  }
  for (int p = 0; p < B; ++p) b->h_tab[p].block = block;   // one width for the whole batch
  BTRY(hipMemcpyAsync(b->d_tab, b->h_tab, sizeof(SweepArgs) * B, hipMemcpyHostToDevice,
                      b->stream));
  // contact data staged in LDS when that costs no extra round of workgroups
  const bool stg = !b->ctx[0]->stage_off &&
                   cd_stage_pick(b->dim, block, lds, lds_stage, b->grid_total, b->grid_total,
                                 b->ctx[0]->num_cu, b->ctx[0]->max_lds, true);
  const size_t lds_launch = stg ? lds_stage : lds;
  b->staged = stg;
  const int every = b->time_every;
  const int groups_cap = every > 0 ? (limit + every - 1) / every : 0;
  if ((int)b->sweep_ev.size() < 2 * groups_cap) {
    size_t old = b->sweep_ev.size();
    b->sweep_ev.resize(2 * (size_t)groups_cap, nullptr);
    for (size_t k = old; k < b->sweep_ev.size(); ++k) BTRY(hipEventCreate(&b->sweep_ev[k]));
  }
  // the launch table: every packing's workgroups; as packings stop, the
  // table is rebuilt without them (their workgroups would only return)
  int grid_now = b->grid_total, stage = 0, live = open;
  BTRY(hipMemcpyAsync(b->d_blk, b->blk_all.data(), sizeof(int) * b->blk_all.size(),
                      hipMemcpyHostToDevice, b->stream));
  BTRY(hipStreamSynchronize(b->stream));
  // each packing's own progress record says when its solve has stopped
  for (int p = 0; p < B; ++p) {
    volatile HostProg* cp = b->ctx[p]->h_prog;
    cp->decided = 0;
    cp->done = 0;
  }
  volatile BatchProg* hp = b->h_prog;
  hp->decided = 0;
  hp->ndone = 0;
  __sync_synchronize();
  const int kLookahead = 8;
  int launched = 0, groups_closed = 0, last_build = 0;
  while (launched < limit && hp->ndone < open) {
    if (launched - last_build >= 16 && open - hp->ndone <= (3 * live) / 4) {
      // compact: keep the packings whose stop has not been published; the
      // copy is ordered after the launches already queued, and a staging
      // buffer is rewritten only 16 or more launches after its last copy,
      // when the lookahead bound guarantees that copy has run
      int* tab = b->h_blk[stage];
      int n2 = 0, still = 0;
      for (int p = 0; p < B; ++p) {
        const cd_ctx* c = b->ctx[p];
        if (b->failed[p] || c->nc == 0 || c->st_limit <= 0 || ((volatile HostProg*)c->h_prog)->done)
          continue;
        ++still;
        const int grid = b->h_tab[p].grid;
        for (int q = 0; q <= grid; ++q) {
          tab[2 * n2] = p;
          tab[2 * n2 + 1] = q;
          ++n2;
        }
      }
      if (n2 > 0) {
        BTRY(hipMemcpyAsync(b->d_blk, tab, sizeof(int) * 2 * (size_t)n2, hipMemcpyHostToDevice,
                            b->stream));
        grid_now = n2;
        stage ^= 1;
      }
      live = still;
      last_build = launched;
    }
    if (launched - hp->decided >= kLookahead) {
      const int seen = hp->decided;
      auto t0 = std::chrono::steady_clock::now();
      while (hp->decided == seen && hp->ndone < open) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
          return bfail(b, CD_EHIP, "batched solve made no progress for 60 s");
      }
      continue;
    }
    const int j = launched + 1;
    const int m = every > 0 && j >= 2 ? (j - 2) / every : -1;
    const bool opens = m >= 0 && (j - 2) % every == 0;
    const bool closes = m >= 0 && (j - 2) % every == every - 1;
    if (opens) BTRY(hipEventRecord(b->sweep_ev[2 * m], b->stream));
    BTRY(cd_launch_sweep_batch(b->stream, b->dim, b->d_tab, b->d_blk, grid_now, block,
                               lds_launch, stg, j, b->d_prog));
    if (closes) {
      BTRY(hipEventRecord(b->sweep_ev[2 * m + 1], b->stream));
      groups_closed = m + 1;
    }
    launched = j;
  }
  // the decisions of the last launched sweep for the packings still open
  BTRY(cd_launch_decide_batch(b->stream, b->d_tab, B, launched, b->d_prog));
  BTRY(cd_launch_gather_states(b->stream, b->d_tab, B, b->d_states));
  BTRY(hipMemcpyAsync(b->h_states, b->d_states, sizeof(SolveState) * B, hipMemcpyDeviceToHost,
                      b->stream));
  BTRY(hipEventRecord(b->ev[2], b->stream));
  BTRY(hipStreamSynchronize(b->stream));
  int max_exec = 0;
  for (int p = 0; p < B; ++p) {
    cd_ctx* c = b->ctx[p];
    if (b->failed[p]) continue;
    memcpy(c->h_state, &b->h_states[p], sizeof(SolveState));
    c->run = SolveRun{};
    c->run.launched = launched;
    c->run.executed = c->nc > 0 ? std::min(launched, c->h_state->iter + 1) : 0;
    max_exec = std::max(max_exec, c->run.executed);
  }
  // ---- every packing's update: launches for all, one synchronisation,
  // then walls, results and timings
  int status = CD_OK;
  BTRY(lanes_after_batch_stream(b));
  lanes_attach(b);
  {
    int st = over_lanes(b, false, [&](int p) { return finish_enqueue(b->ctx[p]); });
    hipError_t e = lanes_sync(b);
    lanes_detach(b);
    if (st != CD_OK) return st;
    if (e != hipSuccess) return bfail(b, CD_EHIP, hipGetErrorString(e));
  }
  BTRY(hipStreamSynchronize(b->stream));
  for (int p = 0; p < B; ++p) {
    if (b->failed[p]) {
      results[p] = cd_result{};
      results[p].status = b->failed[p];
      status = CD_ENONFINITE;
      continue;
    }
    int st = finish_complete(b->ctx[p], &results[p]);
    if (st < 0 && st != CD_ENONFINITE)
      return bfail(b, st, "packing " + std::to_string(p) + ": " + cd_last_error(b->ctx[p]));
    if (st == CD_ENONFINITE) {
      b->failed[p] = CD_ENONFINITE;
      status = CD_ENONFINITE;
    } else if (st == CD_MAXITER && status == CD_OK) {
      status = CD_MAXITER;
    }
  }
  BTRY(hipEventRecord(b->ev[3], b->stream));
  BTRY(hipEventSynchronize(b->ev[3]));
  cd_batch_timing tm{};
  tm.prepare_ms = ms_between(b->ev[0], b->ev[1]);
  tm.solve_ms = ms_between(b->ev[1], b->ev[2]);
  tm.finish_ms = ms_between(b->ev[2], b->ev[3]);
  tm.sweep_launches = launched;
  tm.sweeps_executed = max_exec;
  tm.block_threads = block;
  tm.workgroups = b->grid_total;
  double sum = 0.0;
  int cnt = 0;
  for (int m = 0; m < groups_closed && 2 + (m + 1) * every - 1 <= max_exec; ++m) {
    sum += ms_between(b->sweep_ev[2 * m], b->sweep_ev[2 * m + 1]);
    cnt += every;
  }
  tm.sweep_kernel_ms = cnt > 0 ? sum / cnt * max_exec : 0.0;
  tm.sweeps_timed = cnt;
  tm.staged = b->staged ? 1 : 0;
  b->timing = tm;
  if (status == CD_ENONFINITE) b->err = "some packings diverged and left the batch";
  return status;
}

int cd_batch_get_timing(cd_batch* b, cd_batch_timing* out) {
  if (!b || !out) return CD_EINVAL;
  *out = b->timing;
  return CD_OK;
}

const char* cd_batch_last_error(const cd_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
