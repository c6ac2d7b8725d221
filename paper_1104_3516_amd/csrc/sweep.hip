// sweep.hip - the domain-wise iterative force solve (Sec. 2.1 and 3.1).
//
// One workgroup sweeps one domain.  k_sweep does one sweep per launch (its
// extra workgroup takes the previous sweep's stop decision); k_solve runs all
// sweeps of a step in one launch with a grid barrier after each.  Both give
// the same results.  Per domain and sweep:
//   1. Exchange: recompute the velocities of the domain's particles from
//      their base velocities and external forces plus every incident contact
//      force of the previous sweep (native and foreign), into LDS.  This is
//      the per-sweep exchange of boundary contact forces: other domains'
//      forces are read from the previous sweep's record array.
//   2. Sequential update: colours in order; in a colour, lanes update
//      contacts that share no particle, each solving its own force law with
//      all other forces fixed (Eqs. 3-9, Fig. 2) and applying the change to
//      both bodies' LDS velocities.  A contact's static data (frame,
//      constants, previous force, body pair) is read from memory into
//      registers one colour ahead.  New forces go to the other record array,
//      so no domain sees a force of the current sweep from another domain
//      (foreign contacts stay frozen for the sweep).
//   3. The convergence test values (count passing the relative test,
//      largest change of the others, sum of |R|) are reduced per workgroup.
//  The stop decision reduces the workgroup partials in a fixed order and
//  applies test (I) or (II).
//
// Blocks are mapped to domains so that each of the 8 XCDs (blocks are
// dispatched round-robin over them) works on a contiguous run of domains,
// which are spatial neighbours in the bisection tree and share halo data in
// that XCD's L2.
#include "sweep_core.h"

#include <map>
#include <mutex>
#include <tuple>

namespace {

struct BlockRed {
  long long np[kMaxBlock / 64];
  double md[kMaxBlock / 64], sr[kMaxBlock / 64];
};

// Fixed-order reduction of per-thread test values over the workgroup;
// thread 0 gets the totals.
__device__ inline BlockPartial block_partial(long long npass, double maxd, double sumr,
                                             BlockRed& sh, int nthr) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    npass += __shfl_xor(npass, off, 64);
    double o = __shfl_xor(maxd, off, 64);
    if (o > maxd || o != o) maxd = o;
    sumr += __shfl_xor(sumr, off, 64);
  }
  const int wave = tid >> 6, nw = (nthr + 63) >> 6;
  __syncthreads();
  if ((tid & 63) == 0) {
    sh.np[wave] = npass;
    sh.md[wave] = maxd;
    sh.sr[wave] = sumr;
  }
  __syncthreads();
  BlockPartial p;
  p.n_pass = 0;
  p.max_d_fail = 0.0;
  p.sum_r = 0.0;
  p.pad = 0;
  if (tid == 0) {
    for (int k = 1; k < nw; ++k) {
      npass += sh.np[k];
      if (sh.md[k] > maxd || sh.md[k] != sh.md[k]) maxd = sh.md[k];
      sumr += sh.sr[k];
    }
    p.n_pass = npass;
    p.max_d_fail = maxd;
    p.sum_r = sumr;
  }
  return p;
}

// Convergence test (I) or (II) of sweep j from its reduced test values
// (Sec. 2.1), and the stop decision.  Runs in one thread.
__device__ inline void decide_sweep(const SweepArgs& a, SolveState* st, int j, long long tn,
                                    double tm, double ts) {
  const long long nc = a.nc;
  const double ravg = ts / (double)nc;
  const double prev = st->r_avg;
  int conv;
  if (a.criterion == 0) {
    conv = (10 * tn >= 9 * nc) && (tn == nc || tm < a.alpha * (prev * prev));
  } else {
    double dd = (ravg - prev) * (ravg - prev);
    double ss = (ravg + prev) * (ravg + prev);
    conv = dd < a.alpha * ss || dd == 0.0;
  }
  st->n_pass = tn;
  st->max_d_fail = tm;
  st->r_avg_prev = prev;
  st->r_avg = ravg;
  st->conv = conv;
  st->iter = j;
  if (!isfinite(ts)) {
    st->done = 1;
    st->status = CD_ENONFINITE;
  } else if (a.fixed_iters > 0) {
    if (j >= a.fixed_iters) {
      st->done = 1;
      st->status = CD_OK;
    }
  } else if (conv) {
    st->done = 1;
    st->status = CD_OK;
  } else if (j >= a.max_iter) {
    st->done = 1;
    st->status = CD_MAXITER;
  }
  if (st->done) st->stop_at = j;
}

// Fixed-order reduction of `count` workgroup partials by the calling
// workgroup; thread 0 receives the totals.
__device__ inline BlockPartial reduce_partials(const BlockPartial* part, int count, BlockRed& sh,
                                               int nthr) {
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  for (int q = threadIdx.x; q < count; q += nthr) {
    const BlockPartial p = part[q];
    tn += p.n_pass;
    if (p.max_d_fail > tm || p.max_d_fail != p.max_d_fail) tm = p.max_d_fail;
    ts += p.sum_r;
  }
  return block_partial(tn, tm, ts, sh, nthr);
}

// Stop decision of sweep jd by the calling workgroup: fixed-order reduction
// of that sweep's workgroup partials, test (I) or (II), and the progress
// record for the host.  No-op once the solve is done.
__device__ inline void decide_block(const SweepArgs& a, int jd, BlockRed& red, int& s_flag,
                                    BatchProg* bp, int nthr) {
  SolveState* st = a.state;
  if (threadIdx.x == 0) s_flag = *(volatile const int*)&st->done;
  __syncthreads();
  if (s_flag) return;
  BlockPartial t = reduce_partials(a.partial + (int64_t)(jd & 1) * a.grid, a.grid, red, nthr);
  if (threadIdx.x == 0) {
    decide_sweep(a, st, jd, t.n_pass, t.max_d_fail, t.sum_r);
    __hip_atomic_store(&a.prog->done, st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.prog->decided, jd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (bp) {
      // batched solve: one more packing has stopped
      if (st->done) __hip_atomic_fetch_add(&bp->ndone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&bp->decided, jd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// The same decision taken by one wavefront alone (the calling wave's 64
// lanes): strided fixed-order sums of the partials, then a butterfly.
__device__ inline void decide_wave(const SweepArgs& a, int jd) {
  SolveState* st = a.state;
  const int lane = threadIdx.x & 63;
  int done = 0;
  if (lane == 0) done = *(volatile const int*)&st->done;
  done = __shfl(done, 0, 64);
  if (done) return;
  const BlockPartial* part = a.partial + (int64_t)(jd & 1) * a.grid;
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  // eight partials per lane in flight at once (indices clamped so that the
  // loads are unconditional), then summed in index order
  constexpr int U = 8;
  for (int q0 = lane; q0 < a.grid; q0 += 64 * U) {
    long long np[U];
    double md[U], sr[U];
    for (int u = 0; u < U; ++u) {
      const int q = q0 + 64 * u;
      const BlockPartial* pp = part + (q < a.grid ? q : 0);
      np[u] = pp->n_pass;
      md[u] = pp->max_d_fail;
      sr[u] = pp->sum_r;
    }
    for (int u = 0; u < U; ++u) {
      if (q0 + 64 * u >= a.grid) break;
      tn += np[u];
      if (md[u] > tm || md[u] != md[u]) tm = md[u];
      ts += sr[u];
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    tn += __shfl_xor(tn, off, 64);
    const double o = __shfl_xor(tm, off, 64);
    if (o > tm || o != o) tm = o;
    ts += __shfl_xor(ts, off, 64);
  }
  if (lane == 0) {
    decide_sweep(a, st, jd, tn, tm, ts);
    __hip_atomic_store(&a.prog->done, st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.prog->decided, jd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Sweep j of one domain by workgroup b of a packing's launch, or (b ==
// a.grid) the stop decision of sweep j-1.  A stop at j-1 leaves the forces
// of sweep j-1 final (sweep j writes the other record array); a workgroup
// that already sees the stop skips its domain.
// FOLD (single context, workgroups of two or more wavefronts): there is no
// decision workgroup; the second wavefront of workgroup 0 takes the decision
// while the first updates the colours (or after them when a colour is wider
// than a wavefront), so that a launch has one workgroup per domain.
// TIMED: per-domain load measurement into a.dtick (single contexts with load
// balancing on; a separate instantiation so that the plain sweep is unchanged).
// MOBILE: the box has walls of finite mass (a separate instantiation).
template <int DIM, bool GLOB, bool STAGE, bool FOLD, bool MIXED, bool TIMED, bool RAND,
          bool MOBILE, bool HALO>
__device__ __attribute__((always_inline)) inline void sweep_block(const SweepArgs& a, int b, int j,
                                                                  BatchProg* bp) {
  extern __shared__ double lds[];
  __shared__ BlockRed red;
  __shared__ int s_co[CD_MAX_COLORS + 1];
  __shared__ double s_wu[CD_MAX_WALLS * 3];
  __shared__ double s_wm[MOBILE ? CD_MAX_WALLS : 1];
  __shared__ double s_wtmp[MOBILE ? kMaxBlock : 1];
  __shared__ int s_flag;
  if (!FOLD && b == a.grid) {
    if (j >= 2) decide_block(a, j - 1, red, s_flag, bp, a.block);
    return;
  }
  // the domain's head is read together with the stop flag (one latency)
  const int d = domain_of(a, b, 0, a.grid / 8);
  DomainHead h{};
  if (d >= 0) h = load_head<DIM, STAGE && HALO>(a, d);
  // the decision workgroup may set `done` during this launch: read it once
  if (threadIdx.x == 0) s_flag = *(volatile const int*)&a.state->done;
  __syncthreads();
  if (s_flag) return;
  const double* rin = a.rec[(j - 1) & 1];
  double* rout = a.rec[j & 1];
  long long npass = 0;
  double maxd = 0.0, sumr = 0.0;
  auto idle = [&]() {
    if (FOLD && b == 0 && j >= 2 && (threadIdx.x >> 6) == 1) decide_wave(a, j - 1);
  };
  if (d >= 0) {
    // load measurement (Sec. 3.3): the real-time ticks thread 0 spends on
    // its domain (its wavefront runs the colours; a folded decision is
    // taken by another wavefront and not counted), summed over the step
    const unsigned long long t0 = TIMED ? __builtin_amdgcn_s_memrealtime() : 0ull;
    sweep_domain<DIM, GLOB, STAGE, MIXED, RAND, MOBILE, HALO>(
        a, d, h, rin, rout, lds, s_co, s_wu, npass, maxd, sumr,
        RAND ? rand_mix(a.rkey ^ (unsigned long long)j) : 0ull, idle, s_wm, s_wtmp);
    if (TIMED && threadIdx.x == 0) a.dtick[d] += __builtin_amdgcn_s_memrealtime() - t0;
  } else {
    idle();
  }
  BlockPartial p = block_partial(npass, maxd, sumr, red, a.block);
  if (threadIdx.x == 0) a.partial[(int64_t)(j & 1) * a.grid + b] = p;
}

// Sweep j of one context: a.grid domain workgroups plus its decision workgroup.
// The staged 2D form keeps to 96 VGPRs (five wavefronts per SIMD) so that a
// launch of 2,048 two-wavefront domain workgroups plus the decision
// workgroup is resident at once on 256 CUs.
// MIXED: colour 0 of every domain holds its contacts updated in parallel
// (Sec. 2.3), a separate instantiation so that the plain sweep is unchanged.
// RAND: the random sequential order of Sec. 2.1 (thread 0 of each domain's
// workgroup updates its contacts one at a time), a separate instantiation.
// HALO: the staged form with the foreign incidences' forces in LDS (the
// dynamic LDS of the launch must be sized for it).
template <int DIM, bool GLOB, bool STAGE, bool FOLD, bool MIXED, bool TIMED, bool RAND,
          bool MOBILE, bool HALO>
__global__ __launch_bounds__(kMaxBlock, STAGE && DIM == 2 ? 5 : 1) void k_sweep(SweepArgs a, int j) {
  sweep_block<DIM, GLOB, STAGE, FOLD, MIXED, TIMED, RAND, MOBILE, HALO>(a, blockIdx.x, j, nullptr);
}

// Sweep j of a batch of packings: workgroup b serves packing blk[2b] as its
// workgroup blk[2b+1] (tab holds each packing's arguments).
template <int DIM, bool STAGE>
__global__ __launch_bounds__(kMaxBlock) void k_sweep_batch(const SweepArgs* tab, const int* blk,
                                                          int j, BatchProg* bp) {
  const int2 pb = ((const int2*)blk)[blockIdx.x];
  // read in place: a local copy of the arguments would live in scratch
  const SweepArgs& a = tab[pb.x];
  sweep_block<DIM, false, STAGE, false, false, false, false, false, STAGE>(a, pb.y, j, bp);
}

// stop decision of sweep jd alone (after the last launched sweep)
__global__ __launch_bounds__(kMaxBlock) void k_decide(SweepArgs a, int jd) {
  __shared__ BlockRed red;
  __shared__ int s_flag;
  decide_block(a, jd, red, s_flag, nullptr, kMaxBlock);
}

// the same for every packing of a batch: workgroup p decides packing p
__global__ __launch_bounds__(kMaxBlock) void k_decide_batch(const SweepArgs* tab, int jd,
                                                           BatchProg* bp) {
  __shared__ BlockRed red;
  __shared__ int s_flag;
  const SweepArgs& a = tab[blockIdx.x];
  decide_block(a, jd, red, s_flag, bp, kMaxBlock);
}

// solve states of a batch gathered into one array (one copy to the host)
__global__ __launch_bounds__(64) void k_gather_states(const SweepArgs* tab, int B, SolveState* out) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p < B) out[p] = *tab[p].state;
}

__device__ inline int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p >= target.  Polls are relaxed loads (an acquire per poll
// would invalidate the XCD's L2 under the workgroups still sweeping); the
// caller issues one acquire fence afterwards.  Gives up, raising the abort
// flag, after spin_limit polls so that every wave reaches the kernel's end.
__device__ inline bool wait_at_least(const int* p, int target, GridBar* bar, long long spin_limit) {
  long long spins = 0;
  while (ld_relaxed(p) < target) {
    if (ld_relaxed(&bar->abort)) return false;
    if (++spins > spin_limit) {
      st_release(&bar->abort, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// The whole force solve of one time step in one launch.  All G blocks are
// resident at once (G is sized from the occupancy of this kernel); block b
// runs the domains domain_of(b, k) of its passes k.
// After sweep j every block arrives at a two-level grid barrier (per XCD,
// then across XCDs); the block completing it opens it and owes the stop
// decision of sweep j, which it takes after arriving at barrier j+1, while
// slower blocks are still sweeping.  Past barrier j+1 every block waits for
// that decision: a stop leaves the forces of sweep j final, since sweep j+1
// wrote the other record array.  Every wait is bounded (abort flag).
template <int DIM, bool GLOB>
__global__ __launch_bounds__(kMaxBlock) void k_solve(SweepArgs a, GridBar* bar, int G, int limit,
                                                    long long spin_limit) {
  extern __shared__ double lds[];
  __shared__ BlockRed red;
  __shared__ int s_co[CD_MAX_COLORS + 1];
  __shared__ double s_wu[CD_MAX_WALLS * 3];
  __shared__ int s_last, s_stop;
  SolveState* st = a.state;
  if (*(volatile const int*)&st->done) return;   // nothing to solve: every block returns
  const int b = blockIdx.x, x = b % 8, G8 = G / 8;
  int owe = 0;   // sweep whose decision this block owes (0: none)
  auto decide = [&](int jd) {
    BlockPartial t = reduce_partials(a.partial + (int64_t)(jd & 1) * G, G, red, blockDim.x);
    if (threadIdx.x == 0) {
      if (!__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        decide_sweep(a, st, jd, t.n_pass, t.max_d_fail, t.sum_r);
      st_release(&bar->dec, jd);
    }
  };
  for (int j = 1; j <= limit; ++j) {
    const double* rin = a.rec[(j - 1) & 1];
    double* rout = a.rec[j & 1];
    long long npass = 0;
    double maxd = 0.0, sumr = 0.0;
    for (int k = 0;; ++k) {
      const int d = domain_of(a, b, k, G8);
      if (d < 0) break;
      const DomainHead h = load_head<DIM>(a, d);
      sweep_domain<DIM, GLOB, false>(a, d, h, rin, rout, lds, s_co, s_wu, npass, maxd, sumr,
                                     0ull, [] {});
    }
    BlockPartial p = block_partial(npass, maxd, sumr, red, blockDim.x);
    if (threadIdx.x == 0) {
      a.partial[(int64_t)(j & 1) * G + b] = p;
      // this block's forces and partial, device-wide, before the arrival
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      int last = 0;
      unsigned prev = __hip_atomic_fetch_add(&bar->xcount[x][j & 1], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      if (prev == (unsigned)(G8 - 1)) {
        // last of this XCD: pass the arrivals on
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&bar->xcount[x][j & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev2 = __hip_atomic_fetch_add(&bar->count[j & 1], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        if (prev2 == 7u) {
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
          __hip_atomic_store(&bar->count[j & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st_release(&bar->gen, j);   // barrier j is open
          last = 1;
        }
      }
      s_last = last;
    }
    __syncthreads();
    // the decision this block owes for sweep j-1 (its partials are in the
    // other buffer, untouched until every block has seen that decision)
    if (owe) {
      decide(owe);
      owe = 0;
    }
    if (s_last) owe = j;
    if (threadIdx.x == 0) {
      bool ok = wait_at_least(&bar->gen, j, bar, spin_limit);
      ok = ok && wait_at_least(&bar->dec, j - 1, bar, spin_limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // only a stop decided for a sweep before j counts here: the decision
      // of sweep j may already be out while this block is still at barrier j
      const int stop = __hip_atomic_load(&st->stop_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_stop = !ok || (stop != 0 && stop <= j - 1);
    }
    __syncthreads();
    if (s_stop) break;
  }
  // the decision of the last sweep (at the sweep limit)
  if (owe) decide(owe);
}

// R_avg of the starting forces: kInitBlocks workgroups sum |R| over
// contiguous chunks of the slots, then one workgroup adds the chunk sums in
// order (a fixed reduction order) and resets the solve state.
constexpr int kInitBlocks = 256;

__device__ inline double block_sum_256(double s, double* sh) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  return t;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_rsum(const double* rec0, int64_t nc, double* part) {
  constexpr int REC = cd_rec(DIM);
  __shared__ double sh[4];
  const int64_t chunk = (nc + kInitBlocks - 1) / kInitBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < nc ? lo + chunk : nc;
  double s = 0.0;
  for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    const double* rc = rec0 + q * REC;
    double qq = 0.0;
    for (int k = 0; k < DIM; ++k) qq = qq + rc[k] * rc[k];
    s += sqrt(qq);
  }
  const double t = block_sum_256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_solve_init(const double* part, int64_t nc, SolveState* st,
                                                   int limit, GridBar* bar) {
  __shared__ double sh[4];
  const double t = block_sum_256(threadIdx.x < kInitBlocks ? part[threadIdx.x] : 0.0, sh);
  if (threadIdx.x == 0) {
    for (int x = 0; x < 8; ++x) bar->xcount[x][0] = bar->xcount[x][1] = 0;
    bar->count[0] = bar->count[1] = 0;
    bar->gen = 0;
    bar->dec = 0;
    bar->abort = 0;
    st->iter = 0;
    st->arrive = 0;
    st->n_pass = 0;
    st->max_d_fail = 0.0;
    st->conv = 0;
    st->r_avg = nc > 0 ? t / (double)nc : 0.0;
    st->r_avg_prev = st->r_avg;
    st->stop_at = 0;
    if (nc == 0) {
      st->done = 1;
      st->status = CD_OK;
    } else if (limit <= 0) {
      st->done = 1;
      st->status = CD_MAXITER;
    } else {
      st->done = 0;
      st->status = CD_MAXITER;
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_unslot(const double* rec, const int* contact_slot,
                                               int64_t nc, double* R) {
  constexpr int REC = cd_rec(DIM);
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  const double* rc = rec + (int64_t)contact_slot[c] * REC;
  for (int k = 0; k < DIM; ++k) R[k * nc + c] = rc[k];
}

}  // namespace

SweepArgs cd_sweep_args(cd_ctx* c) {
  SweepArgs a;
  a.dom_start = c->dom_start;
  a.dcol = c->dcol;
  a.dncol = c->dncol;
  a.dp_start = c->dp_start;
  a.gscr = c->gscr;
  a.dpb = c->dpb;
  a.dpe = 2 * c->cap;
  a.dinc_ptr = c->dinc_ptr;
  a.dinc = c->dinc;
  a.ab = c->slot_ab;
  a.geo = c->geo;
  a.walls_u = c->d_wall + (size_t)c->W * c->dim + c->W;
  a.n_walls = c->W;
  a.walls_n = c->d_wall;
  a.walls_dtim = c->d_wall + CD_WALL_DTIM;
  a.walls_force = c->d_wall + CD_WALL_FORCE;
  a.wall_slot = c->wall_slot;
  a.wall_cnt = c->wall_cnt;
  a.mobile = c->mobile_mask;
  a.rec[0] = c->rec[0];
  a.rec[1] = c->rec[1];
  a.ext_zero = (c->ext_fzero ? 1 : 0) | (c->ext_tzero ? 2 : 0);
  a.mu_slot = c->use_mu_slot ? c->mu_slot : c->d_wall + CD_WALL_MU;
  a.mu_step = c->use_mu_slot ? 1 : 0;
  a.state = c->d_state;
  a.partial = c->partial;
  a.prog = c->d_prog;
  a.P = c->P;
  a.n = (int)c->n;
  a.cap = (int)c->cap;
  a.per_xcd = (c->P + 7) / 8;
  a.grid = 8 * a.per_xcd;
  a.block = c->sweep_block;
  a.dtick = c->lb_sigma_star >= 0.0 ? c->d_dtick : nullptr;
  // random sequential order: K = SplitMix64(SplitMix64(seed) ^ step)
  a.rkey = c->order_random ? rand_mix(rand_mix(c->rand_seed) ^ (unsigned long long)c->step) : 0ull;
  a.drow = c->drow;
  a.ddesc = c->ddesc;
  a.halo = c->halo;
  a.hoff = c->hoff;
  a.dhalo = c->dhalo;
  a.hpad = c->hpad;
  a.hstride = c->hstride;
  a.nc = c->nc;
  a.alpha = c->p.alpha;
  a.mu = c->p.mu;
  a.criterion = c->p.criterion;
  a.fixed_iters = c->p.fixed_iters;
  a.max_iter = c->p.max_iter;
  return a;
}

hipError_t cd_launch_solve_init(cd_ctx* c, int limit) {
  if (c->dim == 2)
    hipLaunchKernelGGL(k_rsum<2>, dim3(kInitBlocks), dim3(256), 0, c->stream, c->rec[0], c->nc,
                       c->init_part);
  else
    hipLaunchKernelGGL(k_rsum<3>, dim3(kInitBlocks), dim3(256), 0, c->stream, c->rec[0], c->nc,
                       c->init_part);
  hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(256), 0, c->stream, c->init_part, c->nc,
                     c->d_state, limit, c->d_bar);
  if (c->lb_sigma_star >= 0.0 && c->d_dtick) {
    hipError_t e = hipMemsetAsync(c->d_dtick, 0, sizeof(unsigned long long) * (size_t)c->P,
                                  c->stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// LDS of the random order's draws and ranked slots: 16 bytes reserved per
// contact of the largest domain (an 8-byte draw and a 4-byte rank, padded),
// rounded up to 32 bytes
size_t cd_random_lds(cd_ctx* c) {
  return c->order_random ? ((size_t)16 * std::max(c->st_ds.max_contacts, 1) + 31) / 32 * 32 : 0;
}

static size_t block_lds(cd_ctx* c) {
  return (c->sweep_global ? 0 : (c->sweep_stage ? c->sweep_lds_stage : c->sweep_lds)) +
         cd_random_lds(c);
}

// Workgroups of kernel k resident per CU at this width and dynamic LDS
// (cached: the query is not free and the answer depends only on these).
static int resident_per_cu(const void* k, int block, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_tuple(k, block, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess) n = 0;
  cache[key] = n;
  return n;
}

size_t cd_stage_lds(int max_stage_bytes) {
  const size_t b = (size_t)std::max(max_stage_bytes, 8);
  return (b + 31) / 32 * 32;
}

bool cd_stage_pick(int dim, int block, size_t lds_plain, size_t lds_stage, int64_t wg_stage,
                   int64_t wg_plain, int num_cu, size_t max_lds, bool batch) {
  if (lds_stage + 2048 > max_lds) return false;
  const void* ks;
  const void* kp;
  if (batch) {
    ks = dim == 2 ? (const void*)k_sweep_batch<2, true> : (const void*)k_sweep_batch<3, true>;
    kp = dim == 2 ? (const void*)k_sweep_batch<2, false> : (const void*)k_sweep_batch<3, false>;
  } else {
    ks = dim == 2 ? (const void*)k_sweep<2, false, true, true, false, false, false, false, true>
                  : (const void*)k_sweep<3, false, true, true, false, false, false, false, true>;
    kp = dim == 2 ? (const void*)k_sweep<2, false, false, false, false, false, false, false, false>
                  : (const void*)k_sweep<3, false, false, false, false, false, false, false, false>;
  }
  const int64_t rs = resident_per_cu(ks, block, lds_stage);
  const int64_t rp = resident_per_cu(kp, block, lds_plain);
  if (rs < 1) return false;
  if (rp < 1) return true;
  // staging must not add a round of workgroups
  const int64_t slots_s = rs * num_cu, slots_p = rp * num_cu;
  return (wg_stage + slots_s - 1) / slots_s <= (wg_plain + slots_p - 1) / slots_p;
}

// The plain staged instantiation with the decision folded (no mixed update,
// no load timing, colour-major order, rigid walls), with or without the
// foreign incidences' forces in LDS, for occupancy queries.
static const void* staged_kernel(int dim, bool halo) {
  if (dim == 2)
    return halo ? (const void*)k_sweep<2, false, true, true, false, false, false, false, true>
                : (const void*)k_sweep<2, false, true, true, false, false, false, false, false>;
  return halo ? (const void*)k_sweep<3, false, true, true, false, false, false, false, true>
              : (const void*)k_sweep<3, false, true, true, false, false, false, false, false>;
}

void cd_sweep_mode(cd_ctx* c) {
  c->sweep_stage = false;
  c->sweep_fold = false;
  c->sweep_halo = false;
  if (c->sweep_global || c->stage_off) return;
  const int mu_bytes = c->use_mu_slot ? 8 * c->st_ds.max_contacts : 0;
  // the shared layout needs workgroups at least kUnionMax wide
  const size_t lds_halo = cd_stage_lds(
      (c->sweep_block >= kUnionMax ? c->st_ds.max_stage_u : c->st_ds.max_stage) + mu_bytes);
  const size_t lds_nohalo = cd_stage_lds(c->st_ds.max_stage0 + mu_bytes);
  // With two or more wavefronts per workgroup the decision can fold into
  // workgroup 0.  That pays when a launch runs in several rounds of
  // resident workgroups (a separate decision workgroup would be dispatched
  // last and finish last); when every workgroup is resident at once, the
  // separate decision workgroup runs alongside the domains and workgroup 0
  // would only become the slowest one.
  const int64_t domains = (int64_t)8 * ((c->P + 7) / 8);
  // the random order's draws, and the exchange buffer of walls of finite mass
  // (static LDS beyond the 2 KiB the checks allow for)
  const size_t extra =
      cd_random_lds(c) + (c->mobile_mask ? sizeof(double) * (kMaxBlock + CD_MAX_WALLS) : 0);
  // the foreign incidences' forces staged as well when that saves a round
  // of workgroups, or in 3D when it costs none (their LDS is the price of an
  // exchange that reads nothing from memory; in 2D the plain staged form
  // overlaps its record gathers with the slot staging and was measured
  // faster at equal rounds)
  {
    const void* kh = staged_kernel(c->dim, true);
    const void* kn = staged_kernel(c->dim, false);
    const int64_t rh = lds_halo + extra + 2048 <= c->max_lds
                           ? resident_per_cu(kh, c->sweep_block, lds_halo + extra) * c->num_cu
                           : 0;
    const int64_t rn = resident_per_cu(kn, c->sweep_block, lds_nohalo + extra) * c->num_cu;
    // rounds of resident workgroups for the domain workgroups and the
    // decision workgroup
    const int64_t round_h = rh > 0 ? (domains + rh) / rh : 0;
    const int64_t round_n = rn > 0 ? (domains + rn) / rn : 0;
    c->sweep_halo = rh > 0 && (rn < 1 || round_h < round_n ||
                               (round_h == round_n && c->dim == 3));
  }
  c->sweep_lds_stage = c->sweep_halo ? lds_halo : lds_nohalo;
  c->sweep_stage = cd_stage_pick(c->dim, c->sweep_block, c->sweep_lds + extra,
                                 c->sweep_lds_stage + extra, domains + 1, domains + 1, c->num_cu,
                                 c->max_lds, false);
  if (!c->sweep_stage) c->sweep_halo = false;
  if (c->sweep_stage && c->sweep_block >= 128) {
    const void* kf = staged_kernel(c->dim, c->sweep_halo);
    const int64_t slots =
        (int64_t)resident_per_cu(kf, c->sweep_block, c->sweep_lds_stage + extra) * c->num_cu;
    c->sweep_fold = domains + 1 > slots;
  }
}

// One sweep launch in the context's form (global records, staged with the
// decision folded into workgroup 0, staged, register read-ahead).
template <int DIM, bool MIXED, bool TIMED, bool RAND = false, bool MOBILE = false>
static void launch_sweep_form(cd_ctx* c, const SweepArgs& a, dim3 grid, dim3 block, size_t lds,
                              bool fold, int j) {
  if (c->sweep_global)
    hipLaunchKernelGGL((k_sweep<DIM, true, false, false, MIXED, TIMED, RAND, MOBILE, false>), grid, block,
                       RAND ? lds : 0, c->stream, a, j);
  else if (fold && c->sweep_halo)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, true, MIXED, TIMED, RAND, MOBILE, true>), grid,
                       block, lds, c->stream, a, j);
  else if (fold)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, true, MIXED, TIMED, RAND, MOBILE, false>), grid,
                       block, lds, c->stream, a, j);
  else if (c->sweep_stage && c->sweep_halo)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, false, MIXED, TIMED, RAND, MOBILE, true>), grid,
                       block, lds, c->stream, a, j);
  else if (c->sweep_stage)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, false, MIXED, TIMED, RAND, MOBILE, false>), grid,
                       block, lds, c->stream, a, j);
  else
    hipLaunchKernelGGL((k_sweep<DIM, false, false, false, MIXED, TIMED, RAND, MOBILE, false>), grid,
                       block, lds, c->stream, a, j);
}

template <int DIM>
static void launch_sweep_dim(cd_ctx* c, const SweepArgs& a, dim3 grid, dim3 block, size_t lds,
                             bool fold, int j) {
  const bool timed = a.dtick != nullptr;
  if (c->mobile_mask) {
    // walls of finite mass: the plain colour-major sweep only (the setters
    // refuse the mixed update, the random order and load timing with them)
    launch_sweep_form<DIM, false, false, false, true>(c, a, grid, block, lds, fold, j);
  } else if (c->order_random) {
    launch_sweep_form<DIM, false, false, true>(c, a, grid, block, lds, fold, j);
  } else if (c->order_mixed) {
    if (timed) launch_sweep_form<DIM, true, true>(c, a, grid, block, lds, fold, j);
    else launch_sweep_form<DIM, true, false>(c, a, grid, block, lds, fold, j);
  } else {
    if (timed) launch_sweep_form<DIM, false, true>(c, a, grid, block, lds, fold, j);
    else launch_sweep_form<DIM, false, false>(c, a, grid, block, lds, fold, j);
  }
}

hipError_t cd_launch_sweep(cd_ctx* c, int j, hipEvent_t before, hipEvent_t after) {
  SweepArgs a = cd_sweep_args(c);
  if (before) {
    hipError_t e = hipEventRecord(before, c->stream);
    if (e != hipSuccess) return e;
  }
  // the domain workgroups, plus the decision workgroup unless the decision
  // is folded into workgroup 0
  const bool fold = c->sweep_fold;
  dim3 grid(a.grid + (fold ? 0 : 1)), block(c->sweep_block);
  const size_t lds = block_lds(c);
  if (c->dim == 2) launch_sweep_dim<2>(c, a, grid, block, lds, fold, j);
  else launch_sweep_dim<3>(c, a, grid, block, lds, fold, j);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !after) return e;
  return hipEventRecord(after, c->stream);
}

hipError_t cd_launch_sweep_batch(hipStream_t stream, int dim, const SweepArgs* tab, const int* blk,
                                 int grid, int block, size_t lds, bool stage, int j,
                                 BatchProg* bp) {
  if (dim == 2) {
    if (stage)
      hipLaunchKernelGGL((k_sweep_batch<2, true>), dim3(grid), dim3(block), lds, stream, tab, blk, j, bp);
    else
      hipLaunchKernelGGL((k_sweep_batch<2, false>), dim3(grid), dim3(block), lds, stream, tab, blk, j, bp);
  } else {
    if (stage)
      hipLaunchKernelGGL((k_sweep_batch<3, true>), dim3(grid), dim3(block), lds, stream, tab, blk, j, bp);
    else
      hipLaunchKernelGGL((k_sweep_batch<3, false>), dim3(grid), dim3(block), lds, stream, tab, blk, j, bp);
  }
  return hipGetLastError();
}

hipError_t cd_launch_decide_batch(hipStream_t stream, const SweepArgs* tab, int B, int jd,
                                  BatchProg* bp) {
  if (jd < 1 || B < 1) return hipSuccess;
  hipLaunchKernelGGL(k_decide_batch, dim3(B), dim3(kMaxBlock), 0, stream, tab, jd, bp);
  return hipGetLastError();
}

hipError_t cd_launch_gather_states(hipStream_t stream, const SweepArgs* tab, int B, SolveState* out) {
  if (B < 1) return hipSuccess;
  hipLaunchKernelGGL(k_gather_states, dim3((B + 63) / 64), dim3(64), 0, stream, tab, B, out);
  return hipGetLastError();
}

template <int DIM>
static void launch_sweep_grid_dim(cd_ctx* c, const SweepArgs& a, int j, dim3 g, dim3 block) {
  if (c->sweep_global)
    hipLaunchKernelGGL((k_sweep<DIM, true, false, false, false, false, false, false, false>), g,
                       block, 0, c->stream, a, j);
  else if (c->sweep_stage && c->sweep_halo)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, false, false, false, false, false, true>), g,
                       block, block_lds(c), c->stream, a, j);
  else if (c->sweep_stage)
    hipLaunchKernelGGL((k_sweep<DIM, false, true, false, false, false, false, false, false>), g,
                       block, block_lds(c), c->stream, a, j);
  else
    hipLaunchKernelGGL((k_sweep<DIM, false, false, false, false, false, false, false, false>), g,
                       block, block_lds(c), c->stream, a, j);
}

hipError_t cd_launch_sweep_grid(cd_ctx* c, const SweepArgs& a, int j, int grid) {
  dim3 g(grid), block(c->sweep_block);
  if (c->dim == 2) launch_sweep_grid_dim<2>(c, a, j, g, block);
  else launch_sweep_grid_dim<3>(c, a, j, g, block);
  return hipGetLastError();
}

hipError_t cd_launch_decide(cd_ctx* c, int jd) {
  if (jd < 1) return hipSuccess;
  SweepArgs a = cd_sweep_args(c);
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kMaxBlock), 0, c->stream, a, jd);
  return hipGetLastError();
}

template <int DIM, bool GLOB>
static int solve_capacity(cd_ctx* c) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve<DIM, GLOB>, c->sweep_block,
                                                   block_lds(c)) != hipSuccess)
    return 0;
  return per_cu * c->num_cu;
}

int cd_solve_grid(cd_ctx* c) {
  int cap;
  if (c->dim == 2) cap = c->sweep_global ? solve_capacity<2, true>(c) : solve_capacity<2, false>(c);
  else cap = c->sweep_global ? solve_capacity<3, true>(c) : solve_capacity<3, false>(c);
  const int want = cd_sweep_args(c).grid;
  int g = want < cap ? want : cap;
  return (g / 8) * 8;
}

hipError_t cd_launch_solve(cd_ctx* c, int G, int limit) {
  SweepArgs a = cd_sweep_args(c);
  const long long spin_limit = 1ll << 26;
  dim3 grid(G), block(c->sweep_block);
  if (c->dim == 2) {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_solve<2, true>), grid, block, 0, c->stream, a, c->d_bar, G, limit,
                         spin_limit);
    else
      hipLaunchKernelGGL((k_solve<2, false>), grid, block, block_lds(c), c->stream, a, c->d_bar, G,
                         limit, spin_limit);
  } else {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_solve<3, true>), grid, block, 0, c->stream, a, c->d_bar, G, limit,
                         spin_limit);
    else
      hipLaunchKernelGGL((k_solve<3, false>), grid, block, block_lds(c), c->stream, a, c->d_bar, G,
                         limit, spin_limit);
  }
  return hipGetLastError();
}

hipError_t cd_launch_unslot(cd_ctx* c, int final_iter) {
  if (c->nc == 0) return hipSuccess;
  const double* rec = c->rec[final_iter & 1];
  int nb = cd_blocks(c->nc, 256);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_unslot<2>, dim3(nb), dim3(256), 0, c->stream, rec, c->contact_slot, c->nc,
                       c->R);
  else
    hipLaunchKernelGGL(k_unslot<3>, dim3(nb), dim3(256), 0, c->stream, rec, c->contact_slot, c->nc,
                       c->R);
  return hipGetLastError();
}
