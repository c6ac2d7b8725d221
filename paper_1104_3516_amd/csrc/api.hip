// api.hip - host driver of libcdhip: the C ABI declared in include/cdhip.h.
//
// One time step (the parallel CD scheme of Fig. 7, on one device):
//   boundary width (vmax) -> cell binning -> pair search (canonical list)
//   -> geometry -> warm start -> tree build or descent -> per-domain order
//   -> sweeps until the convergence test holds -> Euler update.
// Host/device synchronisation per step: the vmax readback (the boundary
// width decides the cell search), the contact count (capacity), the domain
// statistics (launch shape), and one state readback per chunk of sweep
// launches (the stop decision itself is taken on the device).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <chrono>
#include <cstdio>

#include "cd_internal.h"

#define CD_TRY(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return e_ == hipErrorOutOfMemory ? CD_ENOMEM : CD_EHIP;                      \
    }                                                                              \
  } while (0)

namespace {

template <typename T>
hipError_t grow(T** p, int64_t count) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  if (count < 1) count = 1;
  return hipMalloc((void**)p, sizeof(T) * (size_t)count);
}

template <typename T>
void release(T** p) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
}

int fail(cd_ctx* c, int code, const std::string& msg);

// ---- workgroup-width tuning (cd_set_launch(ctx, -1)) ----------------------
// The first steps of a context run with the candidate widths in turn; each
// step's mean sweep launch time (HIP events) is recorded and the fastest
// width is kept from then on.  Widths do not change the arithmetic.  The
// choice is cached for the process by (dimension, log2 N, log2 P, device)
// so that later contexts of the same kind start with it.
constexpr int kTuneWidths[4] = {64, 128, 192, 256};

struct TuneKey {
  int dim, nbits, pbits, device;
  bool operator==(const TuneKey& o) const {
    return dim == o.dim && nbits == o.nbits && pbits == o.pbits && device == o.device;
  }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, int>> g_tune_cache;

int ilog2(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

TuneKey tune_key(const cd_ctx* c) { return TuneKey{c->dim, ilog2(c->n), ilog2(c->P), c->device}; }

// the width for the coming solve: a cached choice, the next candidate, or the best seen
int tune_block_pick(cd_ctx* c) {
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (auto& e : g_tune_cache)
      if (e.first == tune_key(c)) {
        c->tune_next = 4;
        c->tune_best = e.second;
        return e.second;
      }
  }
  if (c->tune_next < 4) return kTuneWidths[c->tune_next];
  return c->tune_best > 0 ? c->tune_best : 128;
}

// record the width just used with its mean sweep time
void tune_block_record(cd_ctx* c, double us_per_sweep) {
  if (c->block_override >= 0 || c->tune_next >= 4 || us_per_sweep <= 0.0) return;
  if (c->tune_best == 0 || us_per_sweep < c->tune_best_us) {
    c->tune_best = c->sweep_block;
    c->tune_best_us = us_per_sweep;
  }
  if (++c->tune_next == 4) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache.emplace_back(tune_key(c), c->tune_best);
  }
}
}  // namespace
int cd_fail(cd_ctx* c, int code, const char* msg) { return fail(c, code, msg); }
namespace {
int fail(cd_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

// tree shape of Sec. 3.2 / Fig. 8 for P leaves
void build_tree_shape(cd_ctx* c) {
  const int P = c->P;
  const int nodes = 2 * P - 1;
  c->t_child.assign(2 * nodes, -1);
  c->t_parent.assign(nodes, -1);
  c->t_leaf.assign(nodes, -1);
  c->t_leaves.assign(nodes, 1);
  c->t_level_first.clear();
  c->t_level_count.clear();
  int created = 1;
  if (P > 1) {
    int l = 0;
    while ((1 << (l + 1)) < P) ++l;   // 2^l < P <= 2^(l+1)
    int begin = 0, size = 1;
    auto branch = [&](int node) {
      c->t_child[2 * node] = created;
      c->t_child[2 * node + 1] = created + 1;
      c->t_parent[created] = node;
      c->t_parent[created + 1] = node;
      created += 2;
    };
    for (int m = 0; m < l; ++m) {
      c->t_level_first.push_back(begin);
      c->t_level_count.push_back(size);
      for (int q = 0; q < size; ++q) branch(begin + q);
      begin += size;
      size *= 2;
    }
    int extra = P - (1 << l);
    c->t_level_first.push_back(begin);
    c->t_level_count.push_back(extra);
    for (int q = 0; q < extra; ++q) branch(begin + q);
  }
  // leaves left to right
  std::vector<int> stack;
  stack.push_back(0);
  int next = 0;
  while (!stack.empty()) {
    int node = stack.back();
    stack.pop_back();
    if (c->t_child[2 * node] < 0) {
      c->t_leaf[node] = next++;
    } else {
      stack.push_back(c->t_child[2 * node + 1]);
      stack.push_back(c->t_child[2 * node]);
    }
  }
  for (int node = nodes - 1; node >= 0; --node)
    if (c->t_child[2 * node] >= 0)
      c->t_leaves[node] = c->t_leaves[c->t_child[2 * node]] + c->t_leaves[c->t_child[2 * node + 1]];
  c->h_axis.assign(nodes, -1);
  c->h_cut.assign(nodes, 0.0);
}

int alloc_tree(cd_ctx* c) {
  const int nodes = 2 * c->P - 1;
  CD_TRY(grow(&c->d_child, 2 * nodes));
  CD_TRY(grow(&c->d_leaf, nodes));
  CD_TRY(grow(&c->d_leaves, nodes));
  CD_TRY(grow(&c->d_parent, nodes));
  CD_TRY(grow(&c->d_axis, nodes));
  CD_TRY(grow(&c->d_cut, nodes));
  CD_TRY(grow(&c->d_seg_start, nodes));
  CD_TRY(grow(&c->d_seg_end, nodes));
  CD_TRY(grow(&c->d_nl, nodes));
  CD_TRY(grow(&c->d_region, 6 * (int64_t)(nodes + 1)));
  CD_TRY(hipMemcpy(c->d_child, c->t_child.data(), sizeof(int) * 2 * nodes, hipMemcpyHostToDevice));
  CD_TRY(hipMemcpy(c->d_leaf, c->t_leaf.data(), sizeof(int) * nodes, hipMemcpyHostToDevice));
  CD_TRY(hipMemcpy(c->d_leaves, c->t_leaves.data(), sizeof(int) * nodes, hipMemcpyHostToDevice));
  CD_TRY(hipMemcpy(c->d_parent, c->t_parent.data(), sizeof(int) * nodes, hipMemcpyHostToDevice));
  // per-domain arrays
  const int P = c->P;
  CD_TRY(grow(&c->dom_count, P + 1));
  CD_TRY(grow(&c->dom_start, P + 1));
  CD_TRY(grow(&c->dom_cursor, P + 1));
  CD_TRY(grow(&c->dcol, (int64_t)P * (CD_MAX_COLORS + 1)));
  CD_TRY(grow(&c->dncol, P));
  CD_TRY(grow(&c->dp_count, P + 1));
  CD_TRY(grow(&c->dp_start, P + 1));
  CD_TRY(grow(&c->ddesc, 8 * (int64_t)P));
  CD_TRY(grow(&c->dhalo, (int64_t)P));
  int grid = 8 * ((P + 7) / 8);
  CD_TRY(grow(&c->partial, 2 * grid));   // double-buffered by sweep parity
  c->partial_cap = 2 * grid;
  return CD_OK;
}

// capacity of every contact-sized array except the (ci, cj, R) pair lists
int ensure_capacity(cd_ctx* c, int64_t need) {
  if (need <= c->cap && c->cap > 0) return CD_OK;
  int64_t cap = need + need / 4 + 1024;
  const int rec = cd_rec(c->dim);
  CD_TRY(grow(&c->dom, cap));
  CD_TRY(grow(&c->color, cap));
  CD_TRY(grow(&c->nrm, c->dim * cap));
  CD_TRY(grow(&c->gap, cap));
  CD_TRY(grow(&c->xmid, c->dim * cap));
  for (int k = 0; k < 2; ++k) {
    CD_TRY(grow(&c->sort_keys[k], 2 * cap));
    CD_TRY(grow(&c->sort_vals[k], 2 * cap));
    CD_TRY(grow(&c->rec[k], rec * cap));
  }
  CD_TRY(grow(&c->q_la, cap));
  CD_TRY(grow(&c->q_lb, cap));
  CD_TRY(grow(&c->q_col, cap));
  CD_TRY(grow(&c->q_pos, cap));
  CD_TRY(grow(&c->g_mask, 2 * cap));
  CD_TRY(grow(&c->dpb, (int64_t)(2 * c->dim + 2 * c->dr + 3) * 2 * cap));
  CD_TRY(grow(&c->dinc_ptr, 2 * cap + 1));
  CD_TRY(grow(&c->hoff, 2 * cap + 1));
  CD_TRY(grow(&c->drow, (int64_t)cd_row_width(c->dim) * 2 * cap));
  for (int k = 0; k < 3; ++k) {
    if (k < c->dim) CD_TRY(grow(&c->perm[k], cap));
  }
  CD_TRY(grow(&c->perm_tmp, cap));
  CD_TRY(grow(&c->cnode, cap));
  CD_TRY(grow(&c->side, cap));
  CD_TRY(grow(&c->flag, 2 * cap));
  CD_TRY(grow(&c->flag_scan, 2 * cap + 1));
  CD_TRY(grow(&c->bucket, cap));
  CD_TRY(grow(&c->slot_contact, cap));
  CD_TRY(grow(&c->contact_slot, cap));
  CD_TRY(grow(&c->slot_ab, cap));
  CD_TRY(grow(&c->geo, (int64_t)G_COUNT * cap));
  CD_TRY(grow(&c->dp, 2 * cap));
  CD_TRY(grow(&c->inc, 2 * cap));
  c->cap = cap;
  return CD_OK;
}

int ensure_list(cd_ctx* c, int64_t need, int64_t* cap, int** ci, int** cj, double** R) {
  if (need <= *cap && *cap > 0) return CD_OK;
  int64_t nc = need + need / 4 + 1024;
  CD_TRY(grow(ci, nc));
  CD_TRY(grow(cj, nc));
  CD_TRY(grow(R, c->dim * nc));
  *cap = nc;
  return CD_OK;
}

int setup_grid(cd_ctx* c) {
  double a = 2.2 * c->rmax;
  int64_t total = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < c->dim) {
      double len = c->hi[k] - c->lo[k];
      int64_t m = (int64_t)floor(len / a);
      if (m < 1) m = 1;
      if (m > 4096) m = 4096;
      // a periodic axis needs three cells so that a cell's neighbours are
      // distinct and each pair is seen at one image
      if (c->period[k] > 0.0 && m < 3)
        return fail(c, CD_EINVAL, "a periodic axis must span at least three cells of 2.2 r_max");
      c->ncell[k] = (int)m;
      c->cwidth[k] = len / (double)m;
    } else {
      c->ncell[k] = 1;
      c->cwidth[k] = 1.0;
    }
    total *= c->ncell[k];
  }
  if (total > c->cells_cap) {
    CD_TRY(grow(&c->cell_count, total + 1));
    CD_TRY(grow(&c->cell_start, total + 1));
    c->cells_cap = total;
  }
  c->ncells = total;
  return CD_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0f;
  return ms;
}

}  // namespace

static_assert(sizeof(GridBar) <= 512 && sizeof(DomainStats) <= 512 && 6 * sizeof(double) <= 512,
              "pinned scratch holds every small readback");
static_assert(sizeof(GridBar) <= 8 * kWallSlot && sizeof(DomainStats) <= 8 * kWallSlot &&
                  kWallSlot + CD_MAX_WALLS * 3 <= kSlideSlot && kSlideSlot + 1 == kActiveSlot,
              "the wall velocities and the active-contact count have slots of their own in "
              "the pinned scratch");

extern "C" {

const char* cd_status_string(int s) {
  switch (s) {
    case CD_OK: return "ok";
    case CD_MAXITER: return "sweep cap reached before convergence";
    case CD_EINVAL: return "invalid argument";
    case CD_ENOMEM: return "device allocation failed";
    case CD_ECAPACITY: return "per-domain capacity exceeded";
    case CD_ENONFINITE: return "non-finite value";
    case CD_EHIP: return "HIP runtime error";
    case CD_ENOTREADY: return "particles not set";
    case CD_ESHADOW: return "shadow run differs";
    default: return "unknown status";
  }
}

const char* cd_last_error(const cd_ctx* c) { return c ? c->err.c_str() : "null context"; }

int cd_create(cd_ctx** out, const cd_params* params, int64_t n_particles,
              int64_t contact_capacity, void* stream) {
  if (!out || !params) return CD_EINVAL;
  *out = nullptr;
  if ((params->dim != 2 && params->dim != 3) || n_particles < 1 || params->n_domains < 1 ||
      params->n_walls < 0 || params->n_walls > CD_MAX_WALLS || !(params->dt > 0.0) ||
      n_particles > (int64_t)1 << 30 || contact_capacity < 0 ||
      contact_capacity > (int64_t)1 << 30)
    return CD_EINVAL;
  cd_ctx* c = new cd_ctx();
  c->p = *params;
  if (c->p.repartition_every < 1) c->p.repartition_every = 1;
  c->dim = params->dim;
  c->dr = c->dim == 2 ? 1 : 3;
  c->n = n_particles;
  c->W = params->n_walls;
  c->P = params->n_domains;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return CD_EHIP;
  }
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) ==
            hipSuccess &&
        lds > 0)
      c->max_lds = (size_t)lds;
  }
  const int64_t n = c->n;
  int st = CD_OK;
  auto alloc = [&](double** p, int64_t k) {
    if (st == CD_OK && grow(p, k) != hipSuccess) st = CD_ENOMEM;
  };
  auto alloci = [&](int** p, int64_t k) {
    if (st == CD_OK && grow(p, k) != hipSuccess) st = CD_ENOMEM;
  };
  alloc(&c->x, c->dim * n);
  alloc(&c->v, c->dim * n);
  alloc(&c->w, c->dr * n);
  alloc(&c->r, n);
  alloc(&c->m, n);
  alloc(&c->I, n);
  alloc(&c->f, c->dim * n);
  alloc(&c->t, c->dr * n);
  alloc(&c->inv_m, n);
  alloc(&c->inv_I, n);
  alloc(&c->dtim, n);
  alloc(&c->dtii, n);
  alloc(&c->d_wall, (int64_t)CD_WALL_WORDS);
  alloc(&c->d_wall_new, (int64_t)CD_MAX_WALLS * 3);
  alloci(&c->wall_cnt, CD_MAX_WALLS);
  alloci(&c->cell_of, n);
  alloci(&c->cell_members, n);
  alloc(&c->cell_xr, (c->dim + 1) * n);
  alloci(&c->pair_count, n + 1);
  alloci(&c->pair_off, n + 1);
  alloci(&c->inc_count, n + 1);
  alloci(&c->inc_ptr, n + 1);
  alloci(&c->inc_cursor, n + 1);
  if (st == CD_OK && hipMemcpy(c->d_wall + CD_WALL_MU, &c->p.mu, sizeof(double),
                               hipMemcpyHostToDevice) != hipSuccess)
    st = CD_EHIP;
  if (st == CD_OK && hipMalloc((void**)&c->d_state, sizeof(SolveState)) != hipSuccess) st = CD_ENOMEM;
  if (st == CD_OK) {
    // no solve open until a step sets one up (a batched launch may read it)
    SolveState s0{};
    s0.done = 1;
    if (hipMemcpy(c->d_state, &s0, sizeof(SolveState), hipMemcpyHostToDevice) != hipSuccess)
      st = CD_EHIP;
  }
  if (st == CD_OK && hipMalloc((void**)&c->d_stats, sizeof(DomainStats)) != hipSuccess) st = CD_ENOMEM;
  if (st == CD_OK && hipMemset(c->d_stats, 0, sizeof(DomainStats)) != hipSuccess) st = CD_EHIP;
  if (st == CD_OK && hipMalloc((void**)&c->d_bar, sizeof(GridBar)) != hipSuccess) st = CD_ENOMEM;
  if (st == CD_OK && hipMalloc((void**)&c->init_part, sizeof(double) * 256) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount,
                                            c->device) != hipSuccess ||
                      c->num_cu < 1))
    st = CD_EHIP;
  if (st == CD_OK && hipMalloc((void**)&c->d_vmax, sizeof(unsigned long long)) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipMalloc((void**)&c->d_active, 2 * sizeof(unsigned long long)) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipHostMalloc((void**)&c->h_state, sizeof(SolveState)) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipHostMalloc((void**)&c->h_scratch, 512) != hipSuccess) st = CD_ENOMEM;
  if (st == CD_OK &&
      hipHostMalloc((void**)&c->h_walls, sizeof(double) * CD_WALL_WORDS) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipHostMalloc((void**)&c->h_prog, sizeof(HostProg), hipHostMallocMapped) != hipSuccess)
    st = CD_ENOMEM;
  if (st == CD_OK && hipHostGetDevicePointer((void**)&c->d_prog, c->h_prog, 0) != hipSuccess)
    st = CD_EHIP;
  if (st == CD_OK) {
    build_tree_shape(c);
    st = alloc_tree(c);
  }
  for (int k = 0; k < 8 && st == CD_OK; ++k)
    if (hipEventCreate(&c->ev[k]) != hipSuccess) st = CD_EHIP;
  if (st == CD_OK && hipMemset(c->t, 0, sizeof(double) * c->dr * n) != hipSuccess) st = CD_EHIP;
  if (st == CD_OK && hipMemset(c->f, 0, sizeof(double) * c->dim * n) != hipSuccess) st = CD_EHIP;
  // no wall of finite mass until cd_set_boundary
  if (st == CD_OK && hipMemset(c->d_wall + CD_WALL_DTIM, 0,
                               sizeof(double) * (CD_WALL_WORDS - CD_WALL_DTIM)) != hipSuccess)
    st = CD_EHIP;
  if (st == CD_OK && hipMemset(c->wall_cnt, 0, sizeof(int) * CD_MAX_WALLS) != hipSuccess)
    st = CD_EHIP;
  if (st == CD_OK && contact_capacity > 0) {
    // contact arrays sized up front: both lists of the warm start and every
    // contact-sized workspace
    st = ensure_capacity(c, contact_capacity);
    if (st == CD_OK) st = ensure_list(c, contact_capacity, &c->cap_list, &c->ci, &c->cj, &c->R);
    if (st == CD_OK)
      st = ensure_list(c, contact_capacity, &c->cap_prev, &c->ci_prev, &c->cj_prev, &c->R_prev);
  }
  if (st != CD_OK) {
    cd_destroy(c);
    return st;
  }
  *out = c;
  return CD_OK;
}

int cd_destroy(cd_ctx* c) {
  if (!c) return CD_OK;
  (void)hipDeviceSynchronize();
  double** dbl[] = {&c->x, &c->v, &c->w, &c->r, &c->m, &c->I, &c->f, &c->t, &c->inv_m,
                    &c->inv_I, &c->dtim, &c->dtii, &c->d_wall, &c->nrm, &c->gap, &c->xmid,
                    &c->R, &c->R_prev, &c->d_cut, &c->d_region, &c->geo, &c->rec[0],
                    &c->rec[1], &c->cell_xr};
  for (auto p : dbl) release(p);
  int** ints[] = {&c->cell_of, &c->cell_count, &c->cell_start, &c->cell_members,
                  &c->pair_count, &c->pair_off, &c->ci, &c->cj, &c->dom, &c->color,
                  &c->ci_prev, &c->cj_prev, &c->d_child, &c->d_leaf, &c->d_leaves,
                  &c->d_parent, &c->d_axis, &c->d_seg_start, &c->d_seg_end, &c->d_nl,
                  &c->sort_vals[0], &c->sort_vals[1], &c->perm[0], &c->perm[1], &c->perm[2],
                  &c->perm_tmp, &c->cnode, &c->side, &c->flag, &c->flag_scan, &c->dom_count,
                  &c->dom_start, &c->dom_cursor, &c->bucket, &c->slot_contact,
                  &c->contact_slot, &c->dcol, &c->dncol, &c->dp, &c->dp_count, &c->inc_count,
                  &c->inc_ptr, &c->inc_cursor, &c->inc,
                  &c->dp_start, &c->q_la, &c->q_lb, &c->q_col, &c->q_pos};
  for (auto p : ints) release(p);
  release(&c->sort_keys[0]);
  release(&c->sort_keys[1]);
  release(&c->sort_hist);
  release(&c->scan_tmp);
  release(&c->slot_ab);
  release(&c->g_mask);
  release(&c->gscr);
  release(&c->dpb);
  release(&c->dinc_ptr);
  release(&c->dinc);
  release(&c->drow);
  release(&c->ddesc);
  release(&c->halo);
  release(&c->hpad);
  release(&c->hoff);
  release(&c->dhalo);
  release(&c->d_state);
  release(&c->d_stats);
  release(&c->d_bar);
  release(&c->partial);
  release(&c->init_part);
  release(&c->mu_slot);
  release(&c->ck);
  cd_adjoint_release(c);
  cd_window_clear(c);
  release(&c->d_vmax);
  release(&c->d_active);
  release(&c->d_wall_new);
  release(&c->wall_cnt);
  release(&c->wall_slot);
  release(&c->d_dtick);
  release(&c->par);
  release(&c->d_frac);
  if (c->h_dtick) (void)hipHostFree(c->h_dtick);
  if (c->h_domstart) (void)hipHostFree(c->h_domstart);
  if (c->h_frac) (void)hipHostFree(c->h_frac);
  if (c->h_state) (void)hipHostFree(c->h_state);
  if (c->h_scratch) (void)hipHostFree(c->h_scratch);
  if (c->h_walls) (void)hipHostFree(c->h_walls);
  if (c->h_prog) (void)hipHostFree(c->h_prog);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->sweep_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return CD_OK;
}

int cd_set_particles(cd_ctx* c, const double* x, const double* v, const double* w,
                     const double* radius, const double* mass, const double* inertia) {
  if (!c || !x || !v || !radius || !mass || !inertia) return CD_EINVAL;
  const int64_t n = c->n;
  auto cp = [&](double* dst, const double* src, int64_t k) {
    return hipMemcpyAsync(dst, src, sizeof(double) * (size_t)k, hipMemcpyDeviceToDevice, c->stream);
  };
  CD_TRY(cp(c->x, x, c->dim * n));
  CD_TRY(cp(c->v, v, c->dim * n));
  if (w) CD_TRY(cp(c->w, w, c->dr * n));
  else CD_TRY(hipMemsetAsync(c->w, 0, sizeof(double) * c->dr * n, c->stream));
  CD_TRY(cp(c->r, radius, n));
  CD_TRY(cp(c->m, mass, n));
  CD_TRY(cp(c->I, inertia, n));
  // radii, masses and moments of inertia must be positive and finite
  std::vector<double> h(3 * n);
  CD_TRY(hipMemcpyAsync(h.data(), radius, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  CD_TRY(hipMemcpyAsync(h.data() + n, mass, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  CD_TRY(hipMemcpyAsync(h.data() + 2 * n, inertia, sizeof(double) * n, hipMemcpyDeviceToHost,
                        c->stream));
  CD_TRY(hipStreamSynchronize(c->stream));
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(h[i] > 0.0) || !(h[n + i] > 0.0) || !(h[2 * n + i] > 0.0) || !isfinite(h[i]) ||
        !isfinite(h[n + i]) || !isfinite(h[2 * n + i]))
      return fail(c, CD_EINVAL, "radius, mass and inertia must be positive and finite");
    if (h[i] > rmax) rmax = h[i];
  }
  c->rmax = rmax;
  CD_TRY(cd_launch_derived(c));
  c->have_particles = true;
  c->have_tree = false;
  c->frozen_ready = false;
  c->step = 0;
  c->nc_prev = 0;
  c->list_solved = false;
  c->restored = false;
  return CD_OK;
}

int cd_set_external(cd_ctx* c, const double* force, const double* torque) {
  if (!c) return CD_EINVAL;
  const int64_t n = c->n;
  // whether every force, and every torque, is +0.0 (then the sweeps need not
  // read that part)
  bool zero[2] = {true, true};
  for (int which = 0; which < 2; ++which) {
    const double* src = which == 0 ? force : torque;
    const int64_t count = (which == 0 ? c->dim : c->dr) * n;
    if (!src) continue;
    std::vector<unsigned long long> h((size_t)count);
    CD_TRY(hipMemcpyAsync(h.data(), src, sizeof(double) * (size_t)count, hipMemcpyDeviceToHost,
                          c->stream));
    CD_TRY(hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < count; ++k)
      if (h[(size_t)k] != 0ull) {
        zero[which] = false;
        break;
      }
  }
  c->ext_fzero = zero[0];
  c->ext_tzero = zero[1];
  if (force)
    CD_TRY(hipMemcpyAsync(c->f, force, sizeof(double) * c->dim * n, hipMemcpyDeviceToDevice,
                          c->stream));
  else
    CD_TRY(hipMemsetAsync(c->f, 0, sizeof(double) * c->dim * n, c->stream));
  if (torque)
    CD_TRY(hipMemcpyAsync(c->t, torque, sizeof(double) * c->dr * n, hipMemcpyDeviceToDevice,
                          c->stream));
  else
    CD_TRY(hipMemsetAsync(c->t, 0, sizeof(double) * c->dr * n, c->stream));
  return CD_OK;
}

// Wall normals, offsets and velocities to the device through the pinned
// staging buffer.  sync = false leaves the copy in flight: the caller must
// not change the walls again before the stream has passed it (a time step
// synchronises before its next wall update).
static int upload_walls(cd_ctx* c, bool sync = true) {
  double* buf = c->h_walls;
  const int W = c->W, dim = c->dim;
  for (int k = 0; k < W * dim; ++k) buf[k] = c->wn[k];
  for (int k = 0; k < W; ++k) buf[W * dim + k] = c->wo[k];
  for (int k = 0; k < W * dim; ++k) buf[W * dim + W + k] = c->wu[k];
  // walls of finite mass: dt / M (the same product as in the oracle) and force
  for (int k = 0; k < CD_MAX_WALLS; ++k) {
    buf[CD_WALL_DTIM + k] = k < W ? c->p.dt * c->wim[k] : 0.0;
    buf[CD_WALL_FORCE + k] = k < W ? c->wf[k] : 0.0;
  }
  if (W > 0) {
    CD_TRY(hipMemcpyAsync(c->d_wall, buf, sizeof(double) * (size_t)(W * (2 * dim + 1)),
                          hipMemcpyHostToDevice, c->stream));
    CD_TRY(hipMemcpyAsync(c->d_wall + CD_WALL_DTIM, buf + CD_WALL_DTIM,
                          sizeof(double) * (CD_WALL_WORDS - CD_WALL_DTIM), hipMemcpyHostToDevice,
                          c->stream));
  }
  if (sync) CD_TRY(hipStreamSynchronize(c->stream));
  return CD_OK;
}

int cd_set_walls(cd_ctx* c, const double* normal, const double* offset, const double* velocity) {
  if (!c) return CD_EINVAL;
  const int W = c->W, dim = c->dim;
  if (W > 0 && (!normal || !offset)) return CD_EINVAL;
  for (int k = 0; k < W * dim; ++k) {
    c->wn[k] = normal[k];
    c->wu[k] = velocity ? velocity[k] : 0.0;
  }
  for (int k = 0; k < W; ++k) c->wo[k] = offset[k];
  return upload_walls(c);
}

int cd_set_box(cd_ctx* c, const double* lo, const double* hi) {
  if (!c || !lo || !hi) return CD_EINVAL;
  for (int k = 0; k < 3; ++k) {
    c->lo[k] = k < c->dim ? lo[k] : 0.0;
    c->hi[k] = k < c->dim ? hi[k] : 0.0;
    if (k < c->dim && !(hi[k] > lo[k])) return fail(c, CD_EINVAL, "box must have hi > lo");
    // a periodic axis has the box's length
    c->period[k] = (k < c->dim && ((c->periodic_mask >> k) & 1)) ? c->hi[k] - c->lo[k] : 0.0;
  }
  c->have_box = true;
  return CD_OK;
}

int cd_set_boundary(cd_ctx* c, int periodic_mask, const double* wall_inv_mass,
                    const double* wall_force) {
  if (!c || periodic_mask < 0 || periodic_mask >= (1 << c->dim)) return CD_EINVAL;
  const int W = c->W, dim = c->dim;
  for (int k = 0; k < dim; ++k)
    if ((periodic_mask >> k) & 1)
      for (int q = 0; q < W; ++q)
        if (c->wn[q * dim + k] != 0.0)
          return fail(c, CD_EINVAL, "a wall bounds an axis made periodic");
  int mobile = 0;
  for (int q = 0; q < W; ++q) {
    const double im = wall_inv_mass ? wall_inv_mass[q] : 0.0;
    const double fq = wall_force ? wall_force[q] : 0.0;
    if (!(im >= 0.0) || !std::isfinite(im) || !std::isfinite(fq))
      return fail(c, CD_EINVAL, "wall inverse masses must be >= 0, forces finite");
    if (im != 0.0) mobile |= 1 << q;
  }
  if ((periodic_mask || mobile) && c->adj_every > 0)
    return fail(c, CD_EINVAL, "the adjoint differentiates rigid boxes only");
  if (mobile && (c->mixed_p >= 0.0 || c->order_random || c->lb_sigma_star >= 0.0))
    return fail(c, CD_EINVAL,
                "walls of finite mass go with the plain colour-major sweep only "
                "(no mixed update, random order or load measurement)");
  c->periodic_mask = periodic_mask;
  for (int k = 0; k < 3; ++k)
    c->period[k] = (k < dim && ((periodic_mask >> k) & 1)) ? c->hi[k] - c->lo[k] : 0.0;
  for (int q = 0; q < CD_MAX_WALLS; ++q) {
    c->wim[q] = (wall_inv_mass && q < W) ? wall_inv_mass[q] : 0.0;
    c->wf[q] = (wall_force && q < W) ? wall_force[q] : 0.0;
  }
  c->mobile_mask = mobile;
  c->have_tree = false;
  return upload_walls(c);
}

int cd_set_timing(cd_ctx* c, int every) {
  if (!c || every < 0) return CD_EINVAL;
  c->time_every = every;
  return CD_OK;
}

int cd_set_solve_mode(cd_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 2) return CD_EINVAL;
  c->persistent = mode == 0;
  c->stage_off = mode == 2;
  return CD_OK;
}

int cd_set_load_balance(cd_ctx* c, double sigma_star) {
  if (!c || !std::isfinite(sigma_star)) return CD_EINVAL;
  if (sigma_star >= 0.0 && c->mobile_mask)
    return fail(c, CD_EINVAL, "the load is measured on boxes without walls of finite mass");
  if (sigma_star >= 0.0 && c->order_random)
    return fail(c, CD_EINVAL, "the load is measured on the colour-major sweep only");
  if (sigma_star < 0.0) {
    c->lb_sigma_star = -1.0;
    c->lb_capacity.clear();
    c->lb_have_times = false;
    return CD_OK;
  }
  if (!c->d_dtick) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess ||
        khz <= 0)
      return fail(c, CD_EHIP, "no real-time clock rate");
    c->wall_khz = khz;
    if (hipMalloc((void**)&c->d_dtick, sizeof(unsigned long long) * (size_t)c->P) != hipSuccess)
      return fail(c, CD_ENOMEM, "load measurement buffers");
    if (hipHostMalloc((void**)&c->h_dtick, sizeof(unsigned long long) * (size_t)c->P) !=
            hipSuccess ||
        hipHostMalloc((void**)&c->h_domstart, sizeof(int) * ((size_t)c->P + 1)) != hipSuccess)
      return fail(c, CD_ENOMEM, "load measurement buffers");
  }
  c->lb_sigma_star = sigma_star;
  return CD_OK;
}

int cd_set_domain_capacity(cd_ctx* c, const double* capacity) {
  if (!c) return CD_EINVAL;
  if (!capacity) {
    c->lb_capacity.clear();
    return CD_OK;
  }
  c->lb_capacity.assign(capacity, capacity + c->P);
  return CD_OK;
}

int cd_get_domain_times(cd_ctx* c, double* times_us, double* sigma_t) {
  if (!c) return CD_EINVAL;
  if (!c->lb_have_times) return fail(c, CD_ENOTREADY, "no measured step (cd_set_load_balance)");
  if (times_us) std::copy(c->lb_times.begin(), c->lb_times.end(), times_us);
  if (sigma_t) *sigma_t = c->lb_sigma;
  return CD_OK;
}

int cd_set_launch(cd_ctx* c, int block_threads) {
  if (!c || block_threads < -1 || block_threads > 256 ||
      (block_threads > 0 && block_threads % 64 != 0))
    return CD_EINVAL;
  c->block_override = block_threads;
  c->tune_next = 0;
  c->tune_best_us = 0.0;
  return CD_OK;
}

}  // extern "C"

// A time step runs in three phases: step_prepare (boundary width,
// detection, warm start, partition, order, solve set-up), the solve (one
// context: solve_single; several: the batched solve) and step_finish
// (canonical forces, Euler update, walls, results).
int prep_phase0(cd_ctx* c) {
  if (!c) return CD_EINVAL;
  if (!c->have_particles || !c->have_box) return fail(c, CD_ENOTREADY, "particles or box not set");
  c->adj_valid = false;
  c->prepared = false;
  c->frozen_now = c->frozen && c->frozen_ready;
  // per-contact friction belongs to a list: it lapses when the list is rebuilt
  if (!c->frozen_now) c->use_mu_slot = false;
  if (c->adj_every > 0) {
    // a new step of the adjoint window (the window restarts unless the list is kept)
    if (!c->frozen_now) cd_window_clear(c);
    int st = cd_window_begin(c);
    if (st != CD_OK) return st;
  }
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[0], c->stream));
  if (c->frozen_now) {
    // the kept list: its geometry at the new positions, slot constants, the
    // previous step's forces as warm start, the new base velocities
    CD_TRY(cd_launch_geometry(c));
    if (c->phase_events) CD_TRY(hipEventRecord(c->ev[1], c->stream));
    if (c->phase_events) CD_TRY(hipEventRecord(c->ev[2], c->stream));
    CD_TRY(cd_launch_frozen_refresh(c));
    if (c->phase_events) CD_TRY(hipEventRecord(c->ev[3], c->stream));
    c->st_limit = c->p.fixed_iters > 0 ? c->p.fixed_iters : c->p.max_iter;
    CD_TRY(cd_launch_solve_init(c, c->st_limit));
    c->run = SolveRun{};
    c->prepared = true;
    if (c->adj_every > 0) return cd_window_geometry(c);
    return CD_OK;
  }
  // ---- boundary width 2 vmax dt (Sec. 3.1): the particles' maximum speed
  // stays on the device, where the pair search reads it; the host checks
  // the width with the pair count
  CD_TRY(cd_launch_vmax(c));
  {
    const int dim = c->dim;
    double ws = 0.0;
    for (int wi = 0; wi < c->W; ++wi) {
      double q = 0.0;
      for (int k = 0; k < dim; ++k) q = q + c->wu[wi * dim + k] * c->wu[wi * dim + k];
      const double sp = sqrt(q);
      if (sp > ws) ws = sp;
    }
    c->st_wall_speed = ws;
  }
  // ---- cells and pair count
  int st = setup_grid(c);
  if (st != CD_OK) return st;
  CD_TRY(cd_launch_cells(c));
  CD_TRY(cd_launch_pair_count(c));
  CD_TRY(hipMemcpyAsync(c->h_scratch, c->d_vmax, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                        c->stream));
  CD_TRY(hipMemcpyAsync(c->h_scratch + 1, c->pair_off + c->n, sizeof(int), hipMemcpyDeviceToHost,
                        c->stream));
  return CD_OK;
}

int prep_phase1(cd_ctx* c) {
  if (c->frozen_now) return CD_OK;
  const double dt = c->p.dt;
  double vmax;
  {
    unsigned long long bits = (unsigned long long)c->h_scratch[0];
    memcpy(&vmax, &bits, sizeof(double));
  }
  if (c->st_wall_speed > vmax) vmax = c->st_wall_speed;
  if (!isfinite(vmax)) return fail(c, CD_ENONFINITE, "non-finite velocity");
  const double skin = c->p.skin >= 0.0 ? c->p.skin : 2.0 * vmax * dt;
  c->st_skin = skin;
  if (!(skin <= 0.2 * c->rmax))
    return fail(c, CD_EINVAL, "boundary width exceeds 0.2 r_max (displacement bound)");
  // ---- the previous step's list becomes the warm-start source
  c->restored = false;
  std::swap(c->ci, c->ci_prev);
  std::swap(c->cj, c->cj_prev);
  std::swap(c->R, c->R_prev);
  std::swap(c->cap_prev, c->cap_list);
  c->nc_prev = (c->step > 0 || c->list_solved) ? c->nc : 0;
  const int64_t nc = (int64_t)((int*)(c->h_scratch + 1))[0];
  if (nc < 0 || nc > ((int64_t)1 << 30)) return fail(c, CD_ECAPACITY, "too many contacts");
  int st = ensure_capacity(c, nc);
  if (st != CD_OK) return st;
  st = ensure_list(c, nc, &c->cap_list, &c->ci, &c->cj, &c->R);
  if (st != CD_OK) return st;
  c->nc = nc;
  CD_TRY(cd_launch_pair_fill(c));
  CD_TRY(cd_launch_geometry(c));
  CD_TRY(cd_launch_warm_start(c));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[1], c->stream));
  // ---- partition (Sec. 3.2)
  if (!c->have_tree || c->step % c->p.repartition_every == 0) {
    CD_TRY(cd_launch_orb(c));
    c->have_tree = true;
  } else {
    CD_TRY(cd_launch_descend(c));
  }
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[2], c->stream));
  // ---- order
  CD_TRY(cd_launch_order(c));
  CD_TRY(hipMemcpyAsync(c->h_scratch, c->d_stats, sizeof(DomainStats), hipMemcpyDeviceToHost,
                        c->stream));
  return CD_OK;
}

int prep_phase2(cd_ctx* c) {
  if (c->frozen_now) return CD_OK;
  const int dim = c->dim;
  DomainStats ds;
  memcpy(&ds, c->h_scratch, sizeof(DomainStats));
  if (ds.scan_fault)
    return fail(c, CD_EHIP, "a prefix scan gave up waiting on a predecessor tile");
  if (ds.overflow)
    return fail(c, CD_ECAPACITY,
                ds.overflow == 3 ? "a particle touches contacts of more than 32 domains"
                                 : "a domain needs more than 64 colours");
  if (ds.dinc_total > c->dinc_cap || !c->dinc) {
    int64_t cap = (int64_t)ds.dinc_total + ds.dinc_total / 4 + 1024;
    CD_TRY(grow(&c->dinc, cap));
    // the foreign incidences are a subset of the entries' incidences
    CD_TRY(grow(&c->halo, cap));
    c->dinc_cap = cap;
  }
  {
    // the foreign incidence slots once more at a fixed stride per domain, as
    // many as a sweep workgroup's threads read with the domain's head
    const int64_t stride = std::min<int64_t>(ds.max_halo, 256);
    const int64_t need = stride * (int64_t)c->P;
    if (need > c->hpad_cap || !c->hpad) {
      const int64_t cap = need + need / 4 + 1024;
      CD_TRY(grow(&c->hpad, cap));
      c->hpad_cap = cap;
    }
    c->hstride = (int)stride;
  }
  CD_TRY(cd_launch_order_entries(c));
  // LDS staging per domain, 32-byte aligned; the static LDS of the sweep
  // kernels (colour offsets, reduction scratch) stays below 2 KiB
  const size_t lds = ((size_t)std::max(ds.max_lds, 8) + 31) / 32 * 32;
  // the random order also keeps its draws and ranks in LDS (16 bytes per
  // contact reserved): domains whose records do not fit beside them keep
  // the records in global memory
  const size_t rand_lds =
      c->order_random ? ((size_t)16 * std::max(ds.max_contacts, 1) + 31) / 32 * 32 : 0;
  // walls of finite mass add their exchange buffer to the static LDS
  const size_t mob_lds = c->mobile_mask ? sizeof(double) * (256 + CD_MAX_WALLS) : 0;
  c->sweep_global = lds + rand_lds + mob_lds + 2048 > c->max_lds;
  c->sweep_lds = c->sweep_global ? 0 : lds;
  // one workgroup per domain, wide enough to stage its contacts and gather
  // its particles in one pass (the work is latency-bound)
  {
    // two wavefronts cover the particle gathers of typical domains while
    // keeping every domain's workgroup resident at once; one is enough for
    // small domains
    const int widest = std::max(ds.max_contacts, ds.max_particles);
    c->sweep_block = widest > 64 ? 128 : 64;
    if (c->block_override > 0) c->sweep_block = c->block_override;
    if (c->block_override < 0) c->sweep_block = tune_block_pick(c);
  }
  if (c->sweep_global) {
    // domains too large for LDS stage their data in global memory
    int64_t need = (int64_t)cd_stage_particle(dim) * 2 * c->cap;
    if (need > c->gscr_cap) {
      CD_TRY(grow(&c->gscr, need));
      c->gscr_cap = need;
    }
  }
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[3], c->stream));
  // ---- iterative solve: set-up
  c->st_ds = ds;
  c->st_limit = c->p.fixed_iters > 0 ? c->p.fixed_iters : c->p.max_iter;
  CD_TRY(cd_launch_solve_init(c, c->st_limit));
  c->run = SolveRun{};
  c->prepared = true;
  if (c->frozen) c->frozen_ready = true;
  if (c->adj_every > 0) return cd_window_geometry(c);
  return CD_OK;
}

int step_prepare(cd_ctx* c) {
  int st = prep_phase0(c);
  if (st != CD_OK) return st;
  for (int k = 1; k < kPrepPhases; ++k) {
    CD_TRY(hipStreamSynchronize(c->stream));
    st = prep_phase(c, k);
    if (st != CD_OK) return st;
  }
  return CD_OK;
}

int prep_phase(cd_ctx* c, int k) {
  switch (k) {
    case 0: return prep_phase0(c);
    case 1: return prep_phase1(c);
    case 2: return prep_phase2(c);
  }
  return CD_EINVAL;
}

// Adaptive load balancing (Sec. 3.3) after a measured solve: per-domain
// times in microseconds, their imbalance sigma_T, and, when sigma_T reaches
// the threshold, new capacities (contacts per microsecond; a domain without
// contacts or time gets 0, which the rebuild treats as no measurement)
// that every later tree rebuild uses.
static void lb_after_solve(cd_ctx* c) {
  const int P = c->P;
  const double us_per_tick = 1000.0 / (double)c->wall_khz;
  c->lb_times.assign(P, 0.0);
  double s = 0.0, s2 = 0.0;
  for (int i = 0; i < P; ++i) {
    const double T = (double)c->h_dtick[i] * us_per_tick;
    c->lb_times[i] = T;
    s = s + T;
    s2 = s2 + T * T;
  }
  const double mean = s / (double)P, mean2 = s2 / (double)P;
  double var = mean2 - mean * mean;
  if (var < 0.0) var = 0.0;
  c->lb_sigma = mean > 0.0 ? sqrt(var) / mean : 0.0;
  c->lb_have_times = true;
  if (c->lb_sigma >= c->lb_sigma_star) {
    c->lb_capacity.assign(P, 0.0);
    for (int i = 0; i < P; ++i) {
      const int n = c->h_domstart[i + 1] - c->h_domstart[i];
      const double T = c->lb_times[i];
      c->lb_capacity[i] = (n > 0 && T > 0.0) ? (double)n / T : 0.0;
    }
  }
}

// The solve of one context alone.
int solve_single(cd_ctx* c) {
  const int64_t nc = c->nc;
  const int limit = c->st_limit;
  int launched = 0;
  int executed = -1;
  bool aborted = false;
  bool one_launch = false;
  int groups_closed = 0;
  c->sweep_stage = false;   // the one-launch solve never stages
  c->sweep_fold = false;
  if (c->persistent && c->order_mixed)
    return fail(c, CD_EINVAL, "the one-launch solve has no mixed update (solve modes 1 and 2 do)");
  if (c->persistent && c->order_random)
    return fail(c, CD_EINVAL, "the one-launch solve has no random order (solve modes 1 and 2 do)");
  if (c->persistent && c->mobile_mask)
    return fail(c, CD_EINVAL,
                "the one-launch solve has no walls of finite mass (solve modes 1 and 2 do)");
  const int G = c->persistent ? cd_solve_grid(c) : 0;
  if (G < 8) cd_sweep_mode(c);
  if (c->order_random && nc > 0) {
    const size_t form = c->sweep_global ? 0 : (c->sweep_stage ? c->sweep_lds_stage : c->sweep_lds);
    if (form + cd_random_lds(c) + 2048 > c->max_lds)
      return fail(c, CD_ECAPACITY,
                  "the random order needs 16 bytes of LDS per contact of the largest domain");
  }
  if (G >= 8 && nc > 0 && limit > 0) {
    // all sweeps in one launch
    if ((int)c->sweep_ev.size() < 2) {
      size_t old = c->sweep_ev.size();
      c->sweep_ev.resize(2, nullptr);
      for (size_t k = old; k < 2; ++k) CD_TRY(hipEventCreate(&c->sweep_ev[k]));
    }
    CD_TRY(hipEventRecord(c->sweep_ev[0], c->stream));
    CD_TRY(cd_launch_solve(c, G, limit));
    CD_TRY(hipEventRecord(c->sweep_ev[1], c->stream));
    launched = 1;
    one_launch = true;
    CD_TRY(hipMemcpyAsync(c->h_state, c->d_state, sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    GridBar* hb = (GridBar*)c->h_scratch;
    CD_TRY(hipMemcpyAsync(hb, c->d_bar, sizeof(GridBar), hipMemcpyDeviceToHost, c->stream));
    CD_TRY(hipStreamSynchronize(c->stream));
    aborted = hb->abort != 0;
    // the sweep after the stopping one runs before the stop is seen
    executed = c->h_state->done && c->h_state->iter < limit ? c->h_state->iter + 1 : c->h_state->iter;
  } else if (nc > 0 && limit > 0) {
    // one launch per sweep, queued ahead of the device by at most
    // kLookahead sweeps past the last published decision; launches after
    // the stop return at once.  Progress comes from the mapped record.
    const int kLookahead = 8;
    // timing: launches 2, 3, ... in consecutive groups of `every`, each group
    // bracketed by one pair of events (the first launch carries start-up costs)
    const int every = c->time_every;
    const int groups_cap = every > 0 ? (limit + every - 1) / every : 0;
    if ((int)c->sweep_ev.size() < 2 * groups_cap) {
      size_t old = c->sweep_ev.size();
      c->sweep_ev.resize(2 * (size_t)groups_cap, nullptr);
      for (size_t k = old; k < c->sweep_ev.size(); ++k) CD_TRY(hipEventCreate(&c->sweep_ev[k]));
    }
    groups_closed = 0;
    volatile HostProg* hp = c->h_prog;
    hp->decided = 0;
    hp->done = 0;
    __sync_synchronize();
    // adjoint recording: the forces before the first sweep and after every
    // adj_every-th sweep (fixed sweep count, 2D)
    const bool record = c->adj_every > 0 && c->p.fixed_iters > 0 && c->dim == 2 && !c->win.empty();
    const int64_t rec_bytes = (int64_t)sizeof(double) * 4 * c->cap;
    double* ck = nullptr;
    if (record) {
      cd_ctx::StepRec& r = c->win.back();
      const int64_t slots = limit / c->adj_every + 1;
      CD_TRY(grow(&r.ck, slots * 4 * c->cap));
      CD_TRY(grow(&r.fin, 4 * c->cap));
      ck = r.ck;
      c->ck_stride = 4 * c->cap;
      CD_TRY(hipMemcpyAsync(ck, c->rec[0], rec_bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    while (launched < limit && !hp->done) {
      if (launched - hp->decided >= kLookahead) {
        // wait for the device; give up (CD_EHIP) if it stops making progress
        const int seen = hp->decided;
        auto t0 = std::chrono::steady_clock::now();
        while (hp->decided == seen && !hp->done) {
          if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
            return fail(c, CD_EHIP, "solve made no progress for 60 s");
        }
        continue;
      }
      const int j = launched + 1;
      const int m = every > 0 && j >= 2 ? (j - 2) / every : -1;
      const bool opens = m >= 0 && (j - 2) % every == 0;
      const bool closes = m >= 0 && (j - 2) % every == every - 1;
      CD_TRY(cd_launch_sweep(c, j, opens ? c->sweep_ev[2 * m] : nullptr,
                             closes ? c->sweep_ev[2 * m + 1] : nullptr));
      if (closes) groups_closed = m + 1;
      launched = j;
      if (record && j % c->adj_every == 0)
        CD_TRY(hipMemcpyAsync(ck + (j / c->adj_every) * c->ck_stride, c->rec[j & 1], rec_bytes,
                              hipMemcpyDeviceToDevice, c->stream));
    }
    if (record) {
      cd_ctx::StepRec& r = c->win.back();
      CD_TRY(hipMemcpyAsync(r.fin, c->rec[launched & 1], rec_bytes, hipMemcpyDeviceToDevice,
                            c->stream));
      r.K = launched;
      c->adj_K = launched;
      c->adj_valid = true;
    }
    // the decision of the last launched sweep, if the solve is still open
    CD_TRY(cd_launch_decide(c, launched));
    CD_TRY(hipMemcpyAsync(c->h_state, c->d_state, sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    const bool measure = c->lb_sigma_star >= 0.0 && c->d_dtick && c->P > 0;
    if (measure) {
      CD_TRY(hipMemcpyAsync(c->h_dtick, c->d_dtick, sizeof(unsigned long long) * (size_t)c->P,
                            hipMemcpyDeviceToHost, c->stream));
      CD_TRY(hipMemcpyAsync(c->h_domstart, c->dom_start, sizeof(int) * ((size_t)c->P + 1),
                            hipMemcpyDeviceToHost, c->stream));
    }
    CD_TRY(hipStreamSynchronize(c->stream));
    // sweeps that did work: every launch up to the one after the stopping sweep
    executed = std::min(launched, c->h_state->iter + 1);
    if (measure) lb_after_solve(c);
  } else {
    CD_TRY(hipMemcpyAsync(c->h_state, c->d_state, sizeof(SolveState), hipMemcpyDeviceToHost,
                          c->stream));
    CD_TRY(hipStreamSynchronize(c->stream));
    executed = 0;
  }
  c->run.launched = launched;
  c->run.executed = executed;
  c->run.groups_closed = groups_closed;
  c->run.one_launch = one_launch;
  if (aborted) return fail(c, CD_EHIP, "solve grid barrier did not complete (poll limit)");
  return CD_OK;
}

int finish_enqueue(cd_ctx* c) {
  SolveState s;
  memcpy(&s, c->h_state, sizeof(SolveState));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[4], c->stream));
  // ---- Euler update and canonical forces
  CD_TRY(cd_launch_unslot(c, s.iter));
  CD_TRY(cd_launch_update(c, s.iter));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[5], c->stream));
  CD_TRY(cd_launch_count_active(c, c->d_active));
  CD_TRY(hipMemcpyAsync(c->h_scratch + kSlideSlot, c->d_active, 2 * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, c->stream));
  if (c->mobile_mask) {
    // walls of finite mass: their velocity from the final forces
    CD_TRY(cd_launch_wall_velocities(c));
    CD_TRY(hipMemcpyAsync(c->h_scratch + kWallSlot, c->d_wall_new,
                          sizeof(double) * (size_t)(c->W * c->dim), hipMemcpyDeviceToHost,
                          c->stream));
  }
  return CD_OK;
}

int step_finish(cd_ctx* c, cd_result* out) {
  int st = finish_enqueue(c);
  if (st != CD_OK) return st;
  CD_TRY(hipStreamSynchronize(c->stream));
  return finish_complete(c, out);
}

// The outcome of the last solve and its timings (after the stream has
// passed the finish launches), in c->last, c->timing and *out.
static int collect_result(cd_ctx* c, cd_result* out) {
  const int64_t nc = c->nc;
  const DomainStats& ds = c->st_ds;
  const int launched = c->run.launched, executed = c->run.executed;
  const int groups_closed = c->run.groups_closed;
  const bool one_launch = c->run.one_launch;
  SolveState s;
  memcpy(&s, c->h_state, sizeof(SolveState));
  cd_result res{};
  res.status = nc == 0 ? CD_OK : s.status;
  res.iterations = s.iter;
  res.n_contacts = nc;
  res.n_pass = s.n_pass;
  res.max_d_fail = s.max_d_fail;
  res.r_avg = s.r_avg;
  res.r_avg_prev = s.r_avg_prev;
  res.skin = c->st_skin;
  res.max_colors = ds.max_colors;
  res.max_domain_contacts = ds.max_contacts;
  res.n_active = nc > 0 ? (int64_t)c->h_scratch[kActiveSlot] : 0;
  res.n_sliding = nc > 0 ? (int64_t)c->h_scratch[kSlideSlot] : 0;
  res.crit_last = nc > 0 ? (double)s.n_pass / (double)nc : 1.0;
  {
    const double dd = (s.r_avg - s.r_avg_prev) * (s.r_avg - s.r_avg_prev);
    const double ss = (s.r_avg + s.r_avg_prev) * (s.r_avg + s.r_avg_prev);
    res.rel_change_last = ss > 0.0 ? dd / ss : 0.0;
  }
  c->last = res;
  cd_timing tm{};
  if (c->phase_events) {
    tm.detect_ms = elapsed(c->ev[0], c->ev[1]);
    tm.partition_ms = elapsed(c->ev[1], c->ev[2]);
    tm.order_ms = elapsed(c->ev[2], c->ev[3]);
    tm.solve_ms = elapsed(c->ev[3], c->ev[4]);
    tm.update_ms = elapsed(c->ev[4], c->ev[5]);
  }
  tm.sweep_launches = launched;
  tm.block_threads = c->sweep_block;
  double sk = 0.0;
  tm.sweeps_executed = std::max(executed, 0);
  if (one_launch) {
    sk = elapsed(c->sweep_ev[0], c->sweep_ev[1]);
  } else if (c->time_every > 0 && executed >= 2) {
    // mean launch duration over the closed groups of launches that all did
    // work, times the working sweeps
    const int every = c->time_every;
    double sum = 0.0;
    int cnt = 0;
    for (int m = 0; m < groups_closed && 2 + (m + 1) * every - 1 <= executed; ++m) {
      sum += elapsed(c->sweep_ev[2 * m], c->sweep_ev[2 * m + 1]);
      cnt += every;
    }
    sk = cnt > 0 ? sum / cnt * executed : 0.0;
    tm.sweeps_timed = cnt;
  }
  tm.sweep_kernel_ms = sk;
  tm.staged = c->sweep_stage ? (c->sweep_fold ? 2 : 1) : 0;
  tm.foreign_in_lds = c->sweep_stage && c->sweep_halo ? 1 : 0;
  tm.global_records = c->sweep_global ? 1 : 0;
  c->timing = tm;
  if (c->block_override < 0 && tm.sweeps_timed > 0)
    tune_block_record(c, 1e3 * sk / std::max(executed, 1));
  if (out) *out = res;
  if (res.status == CD_ENONFINITE) return fail(c, CD_ENONFINITE, "non-finite contact force");
  return res.status;
}

int finish_complete(cd_ctx* c, cd_result* out) {
  const int dim = c->dim;
  const double dt = c->p.dt;
  if (c->mobile_mask) {
    const double* U = (const double*)(c->h_scratch + kWallSlot);
    for (int k = 0; k < c->W * dim; ++k) c->wu[k] = U[k];
  }
  // walls move; a box face follows the axis-aligned wall lying on it
  for (int wi = 0; wi < c->W; ++wi) {
    double un = 0.0;
    for (int k = 0; k < dim; ++k) un = un + c->wn[wi * dim + k] * c->wu[wi * dim + k];
    c->wo[wi] = c->wo[wi] + dt * un;
    for (int k = 0; k < dim; ++k) {
      bool unit = true;
      for (int q = 0; q < dim; ++q)
        if (q != k && c->wn[wi * dim + q] != 0.0) unit = false;
      if (!unit) continue;
      if (c->wn[wi * dim + k] == 1.0) c->lo[k] = c->wo[wi];
      if (c->wn[wi * dim + k] == -1.0) c->hi[k] = -c->wo[wi];
    }
  }
  int st = upload_walls(c, false);
  if (st != CD_OK) return st;
  c->step += 1;
  return collect_result(c, out);
}

extern "C" {

int cd_prepare(cd_ctx* c) { return step_prepare(c); }

int cd_set_contact_mu(cd_ctx* c, const double* mu) {
  if (!c || (!mu && c->nc > 0)) return CD_EINVAL;
  if (!c->prepared) return fail(c, CD_ENOTREADY, "cd_set_contact_mu needs cd_prepare first");
  if (c->cap > c->mu_slot_cap) {
    CD_TRY(grow(&c->mu_slot, c->cap));
    c->mu_slot_cap = c->cap;
  }
  CD_TRY(cd_launch_mu_scatter(c, mu));
  c->use_mu_slot = true;
  return CD_OK;
}

int cd_solve(cd_ctx* c, cd_result* out) {
  if (!c) return CD_EINVAL;
  if (!c->prepared) return fail(c, CD_ENOTREADY, "cd_solve needs cd_prepare first");
  c->prepared = false;
  int st = solve_single(c);
  if (st != CD_OK) return st;
  return step_finish(c, out);
}

int cd_set_mixed_update(cd_ctx* c, double p, unsigned long long seed) {
  if (!c || std::isnan(p)) return CD_EINVAL;
  if (p >= 0.0 && c->mobile_mask)
    return fail(c, CD_EINVAL, "walls of finite mass go with the plain sequential update only");
  if (p >= 0.0 && c->adj_every > 0)
    return fail(c, CD_EINVAL, "the adjoint differentiates the sequential update only");
  if (p >= 0.0 && c->order_random)
    return fail(c, CD_EINVAL, "the random order has no parallel contacts");
  c->mixed_p = p >= 0.0 ? p : -1.0;
  c->mixed_seed = seed;
  return CD_OK;
}

int cd_set_random_order(cd_ctx* c, int on, unsigned long long seed) {
  if (!c) return CD_EINVAL;
  if (on && c->mobile_mask)
    return fail(c, CD_EINVAL, "walls of finite mass go with the colour-major order only");
  if (on && c->adj_every > 0)
    return fail(c, CD_EINVAL, "the adjoint differentiates the colour-major order only");
  if (on && c->mixed_p >= 0.0)
    return fail(c, CD_EINVAL, "the random order has no parallel contacts");
  if (on && c->lb_sigma_star >= 0.0)
    return fail(c, CD_EINVAL, "the load is measured on the colour-major sweep only");
  c->order_random = on != 0;
  c->rand_seed = seed;
  return CD_OK;
}

int cd_set_adjoint(cd_ctx* c, int checkpoint_every) {
  if (!c || checkpoint_every < 0) return CD_EINVAL;
  if (checkpoint_every > 0 && c->dim != 2)
    return fail(c, CD_EINVAL, "the adjoint is implemented for 2D");
  if (checkpoint_every > 0 && (c->mobile_mask || c->periodic_mask))
    return fail(c, CD_EINVAL, "the adjoint differentiates rigid boxes only");
  if (checkpoint_every > 0 && c->mixed_p >= 0.0)
    return fail(c, CD_EINVAL, "the adjoint differentiates the sequential update only");
  if (checkpoint_every > 0 && c->order_random)
    return fail(c, CD_EINVAL, "the adjoint differentiates the colour-major order only");
  c->adj_every = checkpoint_every;
  cd_window_clear(c);
  c->adj_valid = false;
  return CD_OK;
}

int cd_set_frozen_list(cd_ctx* c, int on) {
  if (!c) return CD_EINVAL;
  if (on && c->dim != 2) return fail(c, CD_EINVAL, "kept contact lists are implemented for 2D");
  c->frozen = on != 0;
  c->frozen_ready = false;
  return CD_OK;
}

}  // extern "C"

// ---- snapshots: the state a step depends on, between steps
namespace {

struct SnapHeader {
  char magic[8];
  int32_t dim, W, P, flags;   // flags: 1 tree, 2 list of cd_solve_contacts, 4 capacities
  int64_t n, nc, step;
  double wo[CD_MAX_WALLS], wu[CD_MAX_WALLS * 3], lo[3], hi[3];
};
constexpr char kSnapMagic[8] = {'C', 'D', 'S', 'N', 'A', 'P', '1', 0};

int64_t snap_bytes(const cd_ctx* c, int64_t nc, int flags) {
  const int64_t n = c->n, nodes = 2 * (int64_t)c->P - 1;
  int64_t b = (int64_t)sizeof(SnapHeader);
  b += (int64_t)sizeof(double) * (2 * c->dim + c->dr) * n;               // x, v, w
  b += (int64_t)(2 * sizeof(int) + sizeof(double) * c->dim) * nc;        // ci, cj, R
  if (flags & 1) b += (int64_t)(sizeof(int) + sizeof(double)) * nodes;   // axis, cut
  if (flags & 4) b += (int64_t)sizeof(double) * c->P;                    // capacities
  return b;
}

int snap_flags(const cd_ctx* c) {
  return (c->have_tree ? 1 : 0) | (c->list_solved ? 2 : 0) |
         ((int64_t)c->lb_capacity.size() == c->P ? 4 : 0);
}

int snap_check_state(cd_ctx* c) {
  if (c->prepared) return fail(c, CD_ENOTREADY, "snapshots are taken and loaded between steps");
  if (c->frozen || c->adj_every > 0)
    return fail(c, CD_EINVAL, "no snapshots with a kept contact list or the adjoint on");
  return CD_OK;
}

}  // namespace

extern "C" {

int cd_snapshot_size(cd_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return CD_EINVAL;
  *bytes = snap_bytes(c, c->nc, snap_flags(c));
  return CD_OK;
}

int cd_snapshot_save(cd_ctx* c, void* buf, int64_t bytes) {
  if (!c || !buf) return CD_EINVAL;
  int st = snap_check_state(c);
  if (st != CD_OK) return st;
  const int flags = snap_flags(c);
  const int64_t n = c->n, nc = c->nc, nodes = 2 * (int64_t)c->P - 1;
  if (bytes != snap_bytes(c, nc, flags)) return fail(c, CD_EINVAL, "snapshot buffer size");
  SnapHeader hd{};
  memcpy(hd.magic, kSnapMagic, sizeof(kSnapMagic));
  hd.dim = c->dim;
  hd.W = c->W;
  hd.P = c->P;
  hd.flags = flags;
  hd.n = n;
  hd.nc = nc;
  hd.step = c->step;
  memcpy(hd.wo, c->wo, sizeof(hd.wo));
  memcpy(hd.wu, c->wu, sizeof(hd.wu));
  memcpy(hd.lo, c->lo, sizeof(hd.lo));
  memcpy(hd.hi, c->hi, sizeof(hd.hi));
  char* p = (char*)buf;
  memcpy(p, &hd, sizeof(hd));
  p += sizeof(hd);
  auto get = [&](const void* src, size_t nb) {
    hipError_t e = nb ? hipMemcpyAsync(p, src, nb, hipMemcpyDeviceToHost, c->stream) : hipSuccess;
    p += nb;
    return e;
  };
  CD_TRY(get(c->x, sizeof(double) * c->dim * n));
  CD_TRY(get(c->v, sizeof(double) * c->dim * n));
  CD_TRY(get(c->w, sizeof(double) * c->dr * n));
  CD_TRY(get(c->ci, sizeof(int) * nc));
  CD_TRY(get(c->cj, sizeof(int) * nc));
  CD_TRY(get(c->R, sizeof(double) * c->dim * nc));
  if (flags & 1) {
    CD_TRY(get(c->d_axis, sizeof(int) * nodes));
    CD_TRY(get(c->d_cut, sizeof(double) * nodes));
  }
  CD_TRY(hipStreamSynchronize(c->stream));
  if (flags & 4) memcpy(p, c->lb_capacity.data(), sizeof(double) * c->P);
  return CD_OK;
}

int cd_snapshot_load(cd_ctx* c, const void* buf, int64_t bytes) {
  if (!c || !buf) return CD_EINVAL;
  int st = snap_check_state(c);
  if (st != CD_OK) return st;
  if (!c->have_particles || !c->have_box)
    return fail(c, CD_ENOTREADY, "set the particles and the box before loading a snapshot");
  SnapHeader hd;
  if (bytes < (int64_t)sizeof(hd)) return fail(c, CD_EINVAL, "not a snapshot");
  memcpy(&hd, buf, sizeof(hd));
  if (memcmp(hd.magic, kSnapMagic, sizeof(kSnapMagic)) != 0)
    return fail(c, CD_EINVAL, "not a snapshot");
  if (hd.dim != c->dim || hd.W != c->W || hd.P != c->P || hd.n != c->n)
    return fail(c, CD_EINVAL, "snapshot of a context with another dimension, wall, domain "
                              "or particle count");
  if (hd.nc < 0 || hd.step < 0 || bytes != snap_bytes(c, hd.nc, hd.flags))
    return fail(c, CD_EINVAL, "snapshot size");
  const int64_t n = c->n, nc = hd.nc, nodes = 2 * (int64_t)c->P - 1;
  if (hd.flags & 1) {
    // the tree descent indexes positions by the split axes: each inner node's
    // axis must be a coordinate (leaves carry -1)
    const char* ax = (const char*)buf + sizeof(hd) +
                     sizeof(double) * (2 * c->dim + c->dr) * n +
                     (2 * sizeof(int) + sizeof(double) * c->dim) * nc;
    for (int64_t k = 0; k < nodes; ++k) {
      int a;
      memcpy(&a, ax + sizeof(int) * k, sizeof(int));
      const bool inner = c->t_leaf[(size_t)k] < 0;
      if (inner ? (a < 0 || a >= c->dim) : a != -1)
        return fail(c, CD_EINVAL, "snapshot tree with an invalid split axis");
    }
  }
  st = ensure_list(c, nc, &c->cap_list, &c->ci, &c->cj, &c->R);
  if (st == CD_OK) st = ensure_capacity(c, nc);
  if (st != CD_OK) return st;
  const char* p = (const char*)buf + sizeof(hd);
  auto put = [&](void* dst, size_t nb) {
    hipError_t e = nb ? hipMemcpyAsync(dst, p, nb, hipMemcpyHostToDevice, c->stream) : hipSuccess;
    p += nb;
    return e;
  };
  CD_TRY(put(c->x, sizeof(double) * c->dim * n));
  CD_TRY(put(c->v, sizeof(double) * c->dim * n));
  CD_TRY(put(c->w, sizeof(double) * c->dr * n));
  CD_TRY(put(c->ci, sizeof(int) * nc));
  CD_TRY(put(c->cj, sizeof(int) * nc));
  CD_TRY(put(c->R, sizeof(double) * c->dim * nc));
  if (hd.flags & 1) {
    CD_TRY(put(c->d_axis, sizeof(int) * nodes));
    CD_TRY(put(c->d_cut, sizeof(double) * nodes));
  }
  CD_TRY(hipStreamSynchronize(c->stream));
  if (hd.flags & 4) {
    c->lb_capacity.assign((size_t)c->P, 0.0);
    memcpy(c->lb_capacity.data(), p, sizeof(double) * c->P);
  } else {
    c->lb_capacity.clear();
  }
  c->nc = nc;
  c->restored = true;
  c->step = hd.step;
  c->have_tree = (hd.flags & 1) != 0;
  c->list_solved = (hd.flags & 2) != 0;
  memcpy(c->wo, hd.wo, sizeof(hd.wo));
  memcpy(c->wu, hd.wu, sizeof(hd.wu));
  memcpy(c->lo, hd.lo, sizeof(hd.lo));
  memcpy(c->hi, hd.hi, sizeof(hd.hi));
  return upload_walls(c);
}


}  // extern "C"

static int plain_step(cd_ctx* c, cd_result* out) {
  int st = step_prepare(c);
  if (st != CD_OK) return st;
  c->prepared = false;
  st = solve_single(c);
  if (st != CD_OK) return st;
  return step_finish(c, out);
}

namespace {

// The outputs of one step that the shadow run must reproduce.
struct StepOut {
  cd_result r{};
  int64_t nc = 0;
  std::vector<double> d;   // x, v, w, R
  std::vector<int> ij;     // ci, cj
  double wo[CD_MAX_WALLS], wu[CD_MAX_WALLS * 3];
};

int step_outputs(cd_ctx* c, const cd_result& r, StepOut& o) {
  const int64_t n = c->n, nc = c->nc;
  o.r = r;
  o.nc = nc;
  o.d.resize((size_t)((2 * c->dim + c->dr) * n + c->dim * nc));
  o.ij.resize((size_t)(2 * nc));
  double* p = o.d.data();
  auto get = [&](double* dst, const double* src, int64_t k) {
    return k ? hipMemcpyAsync(dst, src, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream)
             : hipSuccess;
  };
  CD_TRY(get(p, c->x, c->dim * n));
  CD_TRY(get(p + c->dim * n, c->v, c->dim * n));
  CD_TRY(get(p + 2 * c->dim * n, c->w, c->dr * n));
  CD_TRY(get(p + (2 * c->dim + c->dr) * n, c->R, c->dim * nc));
  if (nc > 0) {
    CD_TRY(hipMemcpyAsync(o.ij.data(), c->ci, sizeof(int) * nc, hipMemcpyDeviceToHost, c->stream));
    CD_TRY(hipMemcpyAsync(o.ij.data() + nc, c->cj, sizeof(int) * nc, hipMemcpyDeviceToHost,
                          c->stream));
  }
  CD_TRY(hipStreamSynchronize(c->stream));
  memcpy(o.wo, c->wo, sizeof(o.wo));
  memcpy(o.wu, c->wu, sizeof(o.wu));
  return CD_OK;
}

// The first quantity in which two runs of a step differ, or null.
const char* step_difference(const StepOut& a, const StepOut& b) {
  if (a.r.status != b.r.status) return "status";
  if (a.r.iterations != b.r.iterations) return "sweep count";
  if (a.nc != b.nc || a.ij != b.ij) return "contact list";
  const size_t nd = a.d.size();
  if (b.d.size() != nd) return "sizes";
  if (memcmp(a.d.data(), b.d.data(), sizeof(double) * nd) != 0) return "positions, velocities or forces";
  if (memcmp(a.wo, b.wo, sizeof(a.wo)) != 0 || memcmp(a.wu, b.wu, sizeof(a.wu)) != 0) return "walls";
  return nullptr;
}

int shadow_step(cd_ctx* c, cd_result* out) {
  int64_t bytes = 0;
  int st = cd_snapshot_size(c, &bytes);
  if (st != CD_OK) return st;
  std::vector<char> snap((size_t)bytes);
  st = cd_snapshot_save(c, snap.data(), bytes);
  if (st != CD_OK) return st;
  cd_result r1{};
  st = plain_step(c, &r1);
  if (st < 0) return st;
  StepOut first;
  st = step_outputs(c, r1, first);
  if (st != CD_OK) return st;
  if (c->shadow == 2 && c->n > 0) {
    // self-test: the first velocity component moved by 1e-9 (it follows the
    // snapshot header and the positions), enough to survive the rounding of
    // the step's updates
    double v0;
    char* at = snap.data() + sizeof(SnapHeader) + sizeof(double) * c->dim * c->n;
    memcpy(&v0, at, sizeof(double));
    v0 = v0 + 1e-9;
    memcpy(at, &v0, sizeof(double));
  }
  st = cd_snapshot_load(c, snap.data(), bytes);
  if (st != CD_OK) return st;
  cd_result r2{};
  const int st2 = plain_step(c, &r2);
  if (st2 < 0) return st2;
  StepOut second;
  st = step_outputs(c, r2, second);
  if (st != CD_OK) return st;
  const char* diff = step_difference(first, second);
  if (diff)
    return fail(c, CD_ESHADOW, std::string("the shadow run of step ") +
                                   std::to_string(c->step - 1) + " differs in its " + diff);
  if (out) *out = r2;
  return st2;
}

}  // namespace

extern "C" {

int cd_set_shadow(cd_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 2) return CD_EINVAL;
  if (mode && (c->frozen || c->adj_every > 0))
    return fail(c, CD_EINVAL, "no shadow runs with a kept contact list or the adjoint on");
  c->shadow = mode;
  return CD_OK;
}

int cd_step(cd_ctx* c, cd_result* out) {
  if (c && c->shadow) return shadow_step(c, out);
  return plain_step(c, out);
}

int cd_solve_contacts(cd_ctx* c, int64_t n_c, const int32_t* ci, const int32_t* cj,
                      const int32_t* dom, const int32_t* order, double* R_inout,
                      cd_result* out) {
  if (!c) return CD_EINVAL;
  if (!c->have_particles || !c->have_box) return fail(c, CD_ENOTREADY, "particles or box not set");
  if (n_c < 0 || n_c > ((int64_t)1 << 30)) return fail(c, CD_EINVAL, "contact count out of range");
  if (n_c > 0 && (!ci || !cj || !R_inout)) return fail(c, CD_EINVAL, "ci, cj and R are required");
  if (order && !dom) return fail(c, CD_EINVAL, "an update order needs the domains it runs in");
  if (order && (c->mixed_p >= 0.0 || c->order_random))
    return fail(c, CD_EINVAL, "a given update order excludes the mixed update and the random order");
  if (c->adj_every > 0)
    return fail(c, CD_EINVAL, "the adjoint records time steps (cd_step), not cd_solve_contacts");
  c->prepared = false;
  c->adj_valid = false;
  c->frozen_ready = false;
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[0], c->stream));
  // ---- the caller's list becomes the context's current list
  int st = ensure_capacity(c, n_c);
  if (st != CD_OK) return st;
  st = ensure_list(c, n_c, &c->cap_list, &c->ci, &c->cj, &c->R);
  if (st != CD_OK) return st;
  c->nc = n_c;
  c->restored = false;
  c->st_skin = 0.0;
  if (n_c > 0) {
    CD_TRY(hipMemcpyAsync(c->ci, ci, sizeof(int) * (size_t)n_c, hipMemcpyDeviceToDevice, c->stream));
    CD_TRY(hipMemcpyAsync(c->cj, cj, sizeof(int) * (size_t)n_c, hipMemcpyDeviceToDevice, c->stream));
    CD_TRY(hipMemcpyAsync(c->R, R_inout, sizeof(double) * c->dim * (size_t)n_c,
                          hipMemcpyDeviceToDevice, c->stream));
    if (dom)
      CD_TRY(hipMemcpyAsync(c->dom, dom, sizeof(int) * (size_t)n_c, hipMemcpyDeviceToDevice,
                            c->stream));
    // every index is checked before a kernel uses it
    int* fault = &c->d_stats->input_fault;
    CD_TRY(cd_launch_check_inputs(c, dom ? c->dom : nullptr, order, fault));
    CD_TRY(hipMemcpyAsync(c->h_scratch, fault, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CD_TRY(hipStreamSynchronize(c->stream));
    const int bad = ((int*)c->h_scratch)[0];
    if (bad) {
      c->nc = 0;
      return fail(c, CD_EINVAL,
                  (bad & 1) ? "contact list: need 0 <= ci < N, ci < cj < N + W, keys increasing"
                  : (bad & 2) ? "domains must lie in [0, P)"
                              : "order must be a permutation with non-decreasing domains");
    }
  }
  CD_TRY(cd_launch_geometry(c));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[1], c->stream));
  // ---- partition (Sec. 3.2) unless given
  if (!dom) {
    CD_TRY(cd_launch_orb(c));
    c->have_tree = true;
  }
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[2], c->stream));
  // ---- order: colour-major first fit, or the caller's order by levels
  c->given_order = order;
  hipError_t oe = cd_launch_order(c);
  c->given_order = nullptr;
  CD_TRY(oe);
  CD_TRY(hipMemcpyAsync(c->h_scratch, c->d_stats, sizeof(DomainStats), hipMemcpyDeviceToHost,
                        c->stream));
  CD_TRY(hipStreamSynchronize(c->stream));
  const bool frozen = c->frozen;
  c->frozen_now = false;
  c->frozen = false;          // the set-up below must not keep this list for later steps
  st = prep_phase2(c);
  c->frozen = frozen;
  if (st != CD_OK) return st;
  c->prepared = false;
  st = solve_single(c);
  if (st != CD_OK) return st;
  // ---- forces back in canonical order
  SolveState s;
  memcpy(&s, c->h_state, sizeof(SolveState));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[4], c->stream));
  CD_TRY(cd_launch_unslot(c, s.iter));
  if (c->phase_events) CD_TRY(hipEventRecord(c->ev[5], c->stream));
  CD_TRY(cd_launch_count_active(c, c->d_active));
  CD_TRY(hipMemcpyAsync(c->h_scratch + kSlideSlot, c->d_active, 2 * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, c->stream));
  if (n_c > 0)
    CD_TRY(hipMemcpyAsync(R_inout, c->R, sizeof(double) * c->dim * (size_t)n_c,
                          hipMemcpyDeviceToDevice, c->stream));
  CD_TRY(hipStreamSynchronize(c->stream));
  c->list_solved = true;
  return collect_result(c, out);
}

int cd_get_state(cd_ctx* c, double* x, double* v, double* w) {
  if (!c) return CD_EINVAL;
  const int64_t n = c->n;
  if (x) CD_TRY(hipMemcpyAsync(x, c->x, sizeof(double) * c->dim * n, hipMemcpyDeviceToDevice, c->stream));
  if (v) CD_TRY(hipMemcpyAsync(v, c->v, sizeof(double) * c->dim * n, hipMemcpyDeviceToDevice, c->stream));
  if (w) CD_TRY(hipMemcpyAsync(w, c->w, sizeof(double) * c->dr * n, hipMemcpyDeviceToDevice, c->stream));
  CD_TRY(hipStreamSynchronize(c->stream));
  return CD_OK;
}

int cd_get_wall_velocities(cd_ctx* c, double* velocity) {
  if (!c || (!velocity && c->W > 0)) return CD_EINVAL;
  for (int k = 0; k < c->W * c->dim; ++k) velocity[k] = c->wu[k];
  return CD_OK;
}

int cd_get_walls(cd_ctx* c, double* offset) {
  if (!c || (!offset && c->W > 0)) return CD_EINVAL;
  for (int k = 0; k < c->W; ++k) offset[k] = c->wo[k];
  return CD_OK;
}

int64_t cd_num_contacts(const cd_ctx* c) { return c ? c->nc : 0; }

int cd_get_contacts(cd_ctx* c, int64_t cap, int32_t* ci, int32_t* cj, double* normal, double* gap,
                    double* R, int32_t* dom, int32_t* color, int32_t* slot_contact) {
  if (!c) return CD_EINVAL;
  if (c->restored)
    return fail(c, CD_ENOTREADY, "a loaded snapshot holds the warm-start list only: the "
                                 "contacts' data comes with the next step");
  const int64_t nc = c->nc;
  if (cap < nc) return fail(c, CD_EINVAL, "output capacity below the contact count");
  if (nc == 0) return CD_OK;
  auto cpi = [&](int32_t* d, const int* s) {
    return d ? hipMemcpyAsync(d, s, sizeof(int) * nc, hipMemcpyDeviceToDevice, c->stream)
             : hipSuccess;
  };
  auto cpd = [&](double* d, const double* s, int64_t k) {
    return d ? hipMemcpyAsync(d, s, sizeof(double) * k, hipMemcpyDeviceToDevice, c->stream)
             : hipSuccess;
  };
  CD_TRY(cpi(ci, c->ci));
  CD_TRY(cpi(cj, c->cj));
  CD_TRY(cpd(normal, c->nrm, c->dim * nc));
  CD_TRY(cpd(gap, c->gap, nc));
  CD_TRY(cpd(R, c->R, c->dim * nc));
  CD_TRY(cpi(dom, c->dom));
  CD_TRY(cpi(color, c->color));
  CD_TRY(cpi(slot_contact, c->slot_contact));
  CD_TRY(hipStreamSynchronize(c->stream));
  return CD_OK;
}

int cd_get_tree(cd_ctx* c, int32_t* axis, double* cut, int32_t* child, int32_t* leaf) {
  if (!c) return CD_EINVAL;
  const int nodes = 2 * c->P - 1;
  if (axis) CD_TRY(hipMemcpyAsync(axis, c->d_axis, sizeof(int) * nodes, hipMemcpyDeviceToHost, c->stream));
  if (cut) CD_TRY(hipMemcpyAsync(cut, c->d_cut, sizeof(double) * nodes, hipMemcpyDeviceToHost, c->stream));
  CD_TRY(hipStreamSynchronize(c->stream));
  if (child) memcpy(child, c->t_child.data(), sizeof(int) * 2 * nodes);
  if (leaf) memcpy(leaf, c->t_leaf.data(), sizeof(int) * nodes);
  return CD_OK;
}

int cd_get_timing(cd_ctx* c, cd_timing* out) {
  if (!c || !out) return CD_EINVAL;
  *out = c->timing;
  return CD_OK;
}

}  // extern "C"

