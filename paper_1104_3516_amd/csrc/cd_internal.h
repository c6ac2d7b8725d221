// cd_internal.h - context layout and kernel launch wrappers of libcdhip.
//
// Data layout in device memory (FP64 structure-of-arrays unless noted):
//   particles (canonical order i = 0..N-1): x, v (dim x N), w (dr x N), r, m,
//     inertia, f (dim x N), t (dr x N), and the derived 1/m, 1/I, dt/m, dt/I;
//   contacts in canonical (i, j) order: ci, cj, normal (dim x nc), gap,
//     xmid (dim x nc), R (dim x nc, contact frame), dom;
//   contacts in domain-major update order ("slots"): each domain d owns the
//     slot range [dom_start[d], dom_start[d+1]) sorted by (colour, contact id);
//     per slot: local body indices (a, b), frame (n, and t1, t2 in 3D) and the
//     constants of the force law; forces live in two ping-pong record arrays
//     rec[0], rec[1], per slot:
//       2D: (R_n, R_t, F_x, F_y)  with F = R_n n + R_t t the world force,
//       3D: (R_n, R_t1, R_t2, 0, n_x, n_y, n_z, 0); the world force F and
//           the torque per unit lever q = n x R follow from R and the
//           normal with the tangents recomputed from n;
//   per domain: its particles (ascending id) and colour offsets;
//   per particle: incident slots in ascending contact id (sign bit = body 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cdhip.h"

#define CD_MAX_COLORS 64     // colours per domain (64-bit masks)
#define CD_MAX_DC 1024       // contacts per domain
#define CD_MAX_DP 2048       // particles per domain
#define CD_MAX_WALLS 8
// index, in the device wall buffer, of the friction coefficient shared by all contacts
#define CD_WALL_MU (CD_MAX_WALLS * 7)
// then, per wall, dt / M of a wall of finite mass (0: prescribed motion) and
// the external force along its normal
#define CD_WALL_DTIM (CD_WALL_MU + 1)
#define CD_WALL_FORCE (CD_WALL_DTIM + CD_MAX_WALLS)
#define CD_WALL_WORDS (CD_WALL_FORCE + CD_MAX_WALLS)

struct SolveState {
  int iter;           // sweeps completed
  int done;           // 1 once converged, capped or failed
  int status;         // CD_OK, CD_MAXITER or CD_ENONFINITE
  unsigned arrive;    // blocks arrived in the current sweep
  long long n_pass;
  double max_d_fail;
  double r_avg;
  double r_avg_prev;
  int conv;
  int stop_at;        // the sweep whose decision stopped the solve (0: none yet)
};

struct DomainStats {
  int max_colors;
  int max_contacts;
  int max_particles;
  int overflow;       // 2: a domain needs more than CD_MAX_COLORS colours; 3: a particle
                      // touches more than 32 domains
  int max_lds;        // largest per-domain staging size of the sweep, bytes
  int dinc_total;     // incidences summed over all domain particle entries
  int dp_total;       // domain particle entries
  int input_fault;    // a caller's list, domains or order failed the checks (bits 1, 2, 4)
  int max_halo;       // largest count of foreign incidences of a domain
  int max_stage;      // largest staged sweep data of a domain (particles, slots, foreign
                      // incidences), bytes
  int max_stage0;     // the same without the foreign incidences
  int max_stage_u;    // the same with the shared layout for domains of at most kUnionMax
                      // entries
  int scan_fault;     // sticky: a prefix scan gave up waiting on a predecessor tile
                      // (never cleared by the per-step reset of the fields above)
};

// grid barrier of the one-launch solve
struct GridBar {
  unsigned xcount[8][2];  // arrivals per XCD, alternating by sweep parity
  unsigned count[2];      // XCDs whose blocks have all arrived, by parity
  int gen;                // last sweep whose barrier has opened
  int dec;                // last sweep whose stop decision is published
  int abort;              // a wait exceeded its poll limit
  int pad;
};

// progress of the solve, in mapped pinned host memory: written by the
// device (system scope) so the host can follow without synchronising
struct HostProg {
  int decided;        // last sweep whose stop decision is taken
  int done;
  int pad[14];
};

// progress of a batched solve (mapped pinned host memory)
struct BatchProg {
  int decided;        // last sweep whose stop decisions are taken
  int ndone;          // packings whose solve stopped in a decision
  int pad[14];
};

struct BlockPartial {
  long long n_pass;
  double max_d_fail;
  double sum_r;
  long long pad;
};

// Arguments of the sweep kernels (passed by value).
struct SweepArgs {
  // domains
  const int* dom_start;     // P+1 slot offsets
  const int* dcol;          // P x (CD_MAX_COLORS+1) colour offsets inside the domain
  const int* dncol;         // P colours per domain
  const int* dp_start;      // P+1 offsets of the domain particle entries
  double* gscr;             // global stand-in for LDS when a domain does not fit
  // domain particle entries (SoA, stride dpe): v, w, f, t, dt/m, dt/I, r
  const double* dpb;
  int64_t dpe;
  const int* dinc_ptr;      // per entry: incident slots, ascending contact id
  const int* dinc;          // slot * 2 + (1 if body 2)
  const int* drow;          // per entry: the same in fixed-width rows (see k_dinc_rows)
  const int* ddesc;         // per domain: cs, nct, ps, np, ncol (8 ints)
  // foreign incidences (contacts of other domains on the domain's particle
  // entries), listed domain by domain, entry by entry in row order: their
  // slots, each entry's first list index (hoff) and each domain's range
  const int* halo;
  const int* hoff;
  const int2* dhalo;        // per domain: first list index, count
  // the same slots domain by domain at a fixed stride (domain d's first
  // min(count, hstride) of them at d * hstride): read with the head
  const int* hpad;
  int hstride;
  // slots
  const int2* ab;           // local body indices; b < 0: wall -1-b
  const double* geo;        // per-slot constants, SoA with stride cap
  const double* walls_u;    // W x dim wall velocities
  int n_walls;
  double* rec[2];
  int ext_zero;             // bit 0: every external force is +0.0, bit 1: every
                            // external torque is +0.0 (those are then not read)
  const double* mu_slot;    // friction of slot s at mu_slot[s * mu_step]
  int mu_step;              // 1: per slot; 0: one coefficient for all
  // convergence
  SolveState* state;
  BlockPartial* partial;
  HostProg* prog;           // device address of the mapped progress record
  int P;
  int n;                    // particles (SoA stride)
  int cap;                  // slot capacity (SoA stride of geo)
  int grid;                 // blocks of a one-sweep launch
  int block;                // threads per block of a sweep launch
  unsigned long long* dtick;  // per-domain elapsed real-time ticks of the step, or null
  unsigned long long rkey;  // random sequential order: the step's key K (Sec. 2.1)
  // walls of finite mass (Sec. 4.1): normals (W x dim), dt/M and force per
  // wall (device), and each such wall's contact slots in ascending contact
  // id (wall_slot + w * cap, wall_cnt[w] of them)
  const double* walls_n;
  const double* walls_dtim;
  const double* walls_force;
  const int* wall_slot;
  const int* wall_cnt;
  int mobile;               // bit w: wall w has finite mass
  int per_xcd;              // domains per XCD in the block -> domain map
  int wave_lds;             // LDS staging per wavefront (doubles)
  long long nc;
  double alpha;
  double mu;
  int criterion;
  int fixed_iters;
  int max_iter;
};

// Per-slot constants, index k of geo (each block of `cap` doubles):
enum {
  G_N0 = 0,     // normal, dim components
  G_T10 = 3,    // t1 (3D only)
  G_T20 = 6,    // t2 (3D only)
  G_GDT = 9,    // g_e / dt
  G_DWN = 10,   // dt w_n
  G_DWT = 11,   // dt w_t
  G_KN = 12,    // 1 / (dt w_n)
  G_KT = 13,    // 1 / (dt w_t)
  G_COUNT = 14
};

// how the last solve ran (per-sweep launches, timing groups)
struct SolveRun {
  int launched = 0;       // sweep launches (1 for the one-launch solve)
  int executed = 0;       // launches that did work
  int groups_closed = 0;  // complete timing groups of launches
  bool one_launch = false;
};

struct cd_ctx {
  cd_params p{};
  int dim = 2, dr = 1;
  int64_t n = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  bool have_particles = false;
  double rmax = 0.0;
  int64_t step = 0;

  // particles
  double *x = nullptr, *v = nullptr, *w = nullptr, *r = nullptr, *m = nullptr, *I = nullptr;
  double *f = nullptr, *t = nullptr, *inv_m = nullptr, *inv_I = nullptr, *dtim = nullptr,
         *dtii = nullptr;
  // walls (host copies, and a device copy of the velocities)
  int W = 0;
  double wn[CD_MAX_WALLS * 3] = {0}, wo[CD_MAX_WALLS] = {0}, wu[CD_MAX_WALLS * 3] = {0};
  double* d_wall = nullptr;     // normals (W x dim), offsets (W), velocities (W x dim)
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool have_box = false;
  // benchmark boundary conditions (Sec. 4.1, 4.4): periodic axes and walls of
  // finite mass pushed with a constant force
  int periodic_mask = 0;
  double period[3] = {0, 0, 0};   // > 0: periodic axis of this length
  double wim[CD_MAX_WALLS] = {0}, wf[CD_MAX_WALLS] = {0};   // 1/M, force along the normal
  int mobile_mask = 0;            // bit w: wall w has finite mass
  int* wall_slot = nullptr;       // per mobile wall: its contact slots (cap each)
  int* wall_cnt = nullptr;        // their counts (CD_MAX_WALLS)
  int64_t wall_slot_cap = 0;
  double* d_wall_new = nullptr;   // walls' velocities after a step (W x dim)

  // cells
  int ncell[3] = {1, 1, 1};
  double cwidth[3] = {1, 1, 1};
  int64_t ncells = 0, cells_cap = 0;
  int *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_members = nullptr;
  double* cell_xr = nullptr;   // positions and radii in cell order ((dim + 1) x N), pair search

  // contacts (canonical)
  int64_t cap = 0, nc = 0;
  int *pair_count = nullptr, *pair_off = nullptr;
  int *ci = nullptr, *cj = nullptr, *dom = nullptr, *color = nullptr;
  double *nrm = nullptr, *gap = nullptr, *xmid = nullptr, *R = nullptr;
  int64_t cap_list = 0, cap_prev = 0, nc_prev = 0;
  int *ci_prev = nullptr, *cj_prev = nullptr;
  double* R_prev = nullptr;
  double* mu_slot = nullptr;     // per-slot friction of the prepared list (cap)
  int64_t mu_slot_cap = 0;
  bool use_mu_slot = false;      // set by cd_set_contact_mu for the coming solve
  bool prepared = false;         // a step has been prepared and not yet solved
  // frozen contact list: the list, tree and order of the first prepared step
  // are kept for the following steps (geometry recomputed each step)
  bool frozen = false;           // requested by cd_set_frozen_list
  bool frozen_ready = false;     // a list to keep exists
  bool frozen_now = false;       // the step being prepared reuses it
  // adjoint: force checkpoints of the last recorded solve
  int adj_every = 0;             // checkpoint interval in sweeps (0: no recording)
  int adj_K = 0;                 // sweeps of the recorded solve
  bool adj_valid = false;        // the slot data of that solve are still in place
  double* ck = nullptr;          // checkpoints, ck_stride doubles each
  int64_t ck_cap = 0, ck_stride = 0;
  struct AdjointWork* adj = nullptr;  // reverse-pass workspace (adjoint.hip)
  // recorded steps of the adjoint window (one per solve; several only with a
  // frozen list): starting state, geometry, checkpoints, final records
  struct StepRec {
    double* x = nullptr;         // dim x N positions at the step's start
    double* v = nullptr;         // dim x N velocities at the step's start
    double* w = nullptr;         // dr x N
    double* geo_n = nullptr;     // 2 x cap slot normals
    double* geo_gdt = nullptr;   // cap slot g_e/dt
    double* gap = nullptr;       // nc canonical gaps
    double* ck = nullptr;        // checkpoints (S+1) x 4 cap
    double* fin = nullptr;       // final records 4 cap
    int K = 0;                   // sweeps
  };
  std::vector<StepRec> win;

  // tree (host shape + device arrays)
  int P = 1;
  std::vector<int> t_child, t_leaf, t_leaves, t_parent, t_level_first, t_level_count;
  std::vector<int> h_axis;
  std::vector<double> h_cut;
  int* d_child = nullptr;
  int* d_leaf = nullptr;
  int* d_leaves = nullptr;
  int* d_parent = nullptr;
  int* d_axis = nullptr;
  double* d_cut = nullptr;
  int *d_seg_start = nullptr, *d_seg_end = nullptr, *d_nl = nullptr;
  double* d_region = nullptr;   // (2P-1) x 6: lo[3], hi[3]
  bool have_tree = false;
  // ORB workspace (cap-sized)
  unsigned long long* sort_keys[2] = {nullptr, nullptr};
  int* sort_vals[2] = {nullptr, nullptr};
  int* perm[3] = {nullptr, nullptr, nullptr};
  int* perm_tmp = nullptr;
  int* cnode = nullptr;
  int* side = nullptr;
  int* flag = nullptr;
  int* flag_scan = nullptr;
  unsigned* sort_hist = nullptr;
  int64_t sort_hist_cap = 0;

  // order / slots
  int *dom_count = nullptr, *dom_start = nullptr, *dom_cursor = nullptr, *bucket = nullptr;
  int *slot_contact = nullptr, *contact_slot = nullptr;
  int2* slot_ab = nullptr;
  double* geo = nullptr;
  double* rec[2] = {nullptr, nullptr};
  bool ext_fzero = true;         // every external force is +0.0
  bool ext_tzero = true;         // every external torque is +0.0
  int *dcol = nullptr, *dncol = nullptr, *dp = nullptr, *dp_count = nullptr, *dp_start = nullptr;
  int *q_la = nullptr, *q_lb = nullptr, *q_col = nullptr, *q_pos = nullptr;
  unsigned long long* g_mask = nullptr;
  double* gscr = nullptr;
  int64_t gscr_cap = 0;
  double* dpb = nullptr;         // domain particle entries, SoA with stride 2 cap
  int* dinc_ptr = nullptr;       // 2 cap + 1
  int* dinc = nullptr;
  int64_t dinc_cap = 0;
  int* drow = nullptr;           // 2 cap x row width
  int* ddesc = nullptr;          // P x 8
  int* halo = nullptr;           // foreign incidence slots (capacity dinc_cap)
  int* hoff = nullptr;           // 2 cap + 1: per entry, first foreign incidence
  int2* dhalo = nullptr;         // P: per domain, first foreign incidence and count
  int* hpad = nullptr;           // P x hstride: each domain's first foreign incidence slots
  int64_t hpad_cap = 0;
  int hstride = 0;
  int sweep_block = 64;          // threads per domain workgroup
  int block_override = 0;        // 0: chosen from the domain sizes; -1: tuned
  int tune_next = 0;             // next candidate width to try (4: tuning over)
  int tune_best = 0;             // fastest width seen
  double tune_best_us = 0.0;     // its mean sweep launch time
  bool sweep_global = false;
  size_t max_lds = 65536;
  int *inc_count = nullptr, *inc_ptr = nullptr, *inc_cursor = nullptr, *inc = nullptr;
  DomainStats* d_stats = nullptr;

  // solve
  SolveState* d_state = nullptr;
  GridBar* d_bar = nullptr;
  int num_cu = 0;
  bool persistent = false;  // one launch per solve (grid barrier) instead of per sweep
  SolveState* h_state = nullptr;   // pinned
  HostProg* h_prog = nullptr;      // mapped pinned (host address)
  HostProg* d_prog = nullptr;      // its device address
  int time_every = 1;              // sweep launches timed with events: every k-th (0: none)
  bool phase_events = true;        // events around the step's phases (off while in a batch)
  BlockPartial* partial = nullptr;
  double* init_part = nullptr;     // chunk sums of |R| at the start of a solve (256)
  int partial_cap = 0;
  unsigned long long* d_vmax = nullptr;
  long long* h_scratch = nullptr;  // pinned small readbacks
  double* h_walls = nullptr;       // pinned staging of the wall upload

  // scan workspace
  unsigned long long* scan_tmp = nullptr;  // ticket counter, then per-tile status words
  int64_t scan_tmp_cap = 0;                // status words
  uint64_t scan_epoch = 0;                 // scans issued on this context

  // sweep launch shape
  size_t sweep_lds = 0;     // LDS staging per wavefront (domain), bytes
  size_t sweep_lds_stage = 0;  // the same with the domain's contact data staged too
  bool sweep_stage = false;    // this solve stages contact data in LDS
  bool sweep_fold = false;     // ... and takes the stop decision in workgroup 0
  bool sweep_halo = false;     // ... and stages the foreign incidences' forces too
  bool stage_off = false;      // never stage (the register read-ahead form only)

  // timing
  hipEvent_t ev[8] = {};
  std::vector<hipEvent_t> sweep_ev;
  cd_timing timing{};
  cd_result last{};
  // cd_solve_contacts: the caller's update order (device, during the call only)
  const int* given_order = nullptr;
  bool list_solved = false;    // the current list holds forces of cd_solve_contacts
  int shadow = 0;              // cd_set_shadow mode
  bool restored = false;       // the list came from a snapshot: only ci, cj, R are its own
  unsigned long long* d_active = nullptr;   // sliding, closed contacts after the last solve
  // the current step, between its phases
  double st_skin = 0.0;
  double st_wall_speed = 0.0;   // largest wall speed of the step (host)

  // mixed sequential/parallel update (Sec. 2.3)
  double mixed_p = -1.0;                // share of contacts updated in parallel; < 0: none
  unsigned long long mixed_seed = 0;
  unsigned char* par = nullptr;         // per contact: updated in parallel
  int64_t par_cap = 0;
  bool order_mixed = false;             // the current order has a parallel colour 0
  bool order_random = false;            // random sequential order in every sweep (Sec. 2.1)
  unsigned long long rand_seed = 0;

  // adaptive load balancing (Sec. 3.3)
  double lb_sigma_star = -1.0;          // threshold on sigma_T; < 0: no measurement
  std::vector<double> lb_capacity;      // capacities of the tree rebuilds (empty: leaf counts)
  std::vector<double> lb_times;         // last step's per-domain sweep times, microseconds
  double lb_sigma = 0.0;                // their sigma_T
  bool lb_have_times = false;
  int wall_khz = 0;                     // real-time counter frequency
  unsigned long long* d_dtick = nullptr;   // per-domain ticks (P)
  unsigned long long* h_dtick = nullptr;   // pinned copies of them and of the domain
  int* h_domstart = nullptr;               // contact offsets (P + 1)
  double* d_frac = nullptr;             // left-branch shares of the nodes (2P-1)
  double* h_frac = nullptr;             // pinned staging of them
  DomainStats st_ds{};
  int st_limit = 0;
  SolveRun run;
};

// phases of a time step (api.hip); the batch runs them for several contexts
int step_prepare(cd_ctx* c);
// step_prepare in kPrepPhases parts; each part but the last ends with a small
// device-to-host copy that the next part reads, so the caller synchronises
// the stream between parts (once for a whole batch)
constexpr int kPrepPhases = 3;
int prep_phase(cd_ctx* c, int k);
int solve_single(cd_ctx* c);
int step_finish(cd_ctx* c, cd_result* out);
// step_finish in two parts: the update launches, then (after the stream has
// passed them) the walls, results and timings
int finish_enqueue(cd_ctx* c);
int finish_complete(cd_ctx* c, cd_result* out);
int cd_fail(cd_ctx* c, int code, const char* msg);

// ---- launch wrappers (each enqueues on ctx->stream) -----------------------
// scan.hip
hipError_t cd_scan_exclusive(cd_ctx* c, const int* in, int* out, int64_t n);
// sort.hip: stable LSD radix sort of (key, value) pairs, `bits` low key bits
hipError_t cd_radix_sort(cd_ctx* c, unsigned long long* keys, int* vals, unsigned long long* keys_tmp,
                         int* vals_tmp, int64_t n, int bits, unsigned long long** keys_out,
                         int** vals_out);
// detect.hip
hipError_t cd_launch_vmax(cd_ctx* c);
hipError_t cd_launch_cells(cd_ctx* c);
hipError_t cd_launch_pair_count(cd_ctx* c);   // boundary width from d_vmax and st_wall_speed
hipError_t cd_launch_pair_fill(cd_ctx* c);
hipError_t cd_launch_geometry(cd_ctx* c);
hipError_t cd_launch_warm_start(cd_ctx* c);
// partition.hip
hipError_t cd_launch_orb(cd_ctx* c);
hipError_t cd_launch_descend(cd_ctx* c);
// order.hip
hipError_t cd_launch_order(cd_ctx* c);
hipError_t cd_launch_order_entries(cd_ctx* c);   // after the stats readback
// checks of a caller's list (c->ci, c->cj, c->nc), domains and order before use
hipError_t cd_launch_check_inputs(cd_ctx* c, const int* dom, const int* order, int* fault);
// sweep.hip
hipError_t cd_launch_solve_init(cd_ctx* c, int limit);
// sweep j; its extra workgroup takes the stop decision of sweep j-1
hipError_t cd_launch_sweep(cd_ctx* c, int j, hipEvent_t before, hipEvent_t after);
hipError_t cd_launch_decide(cd_ctx* c, int jd);            // stop decision of sweep jd alone
// sweep j with explicit arguments and only the domain workgroups (no decision)
hipError_t cd_launch_sweep_grid(cd_ctx* c, const SweepArgs& a, int j, int grid);
// batched solve over the packings of tab (device array of their arguments)
hipError_t cd_launch_sweep_batch(hipStream_t stream, int dim, const SweepArgs* tab, const int* blk,
                                 int grid, int block, size_t lds, bool stage, int j,
                                 BatchProg* bp);
// LDS of the staged sweep for domains of these sizes (particle entries,
// contacts), with the context's friction mode
size_t cd_stage_lds(int max_stage_bytes);
// LDS of the random order's draws and ranked slots per workgroup (0 without it)
size_t cd_random_lds(cd_ctx* c);
// whether a launch of `workgroups` should stage contact data: it must fit and
// must not need more rounds of resident workgroups than the register form
bool cd_stage_pick(int dim, int block, size_t lds_plain, size_t lds_stage, int64_t wg_stage,
                   int64_t wg_plain, int num_cu, size_t max_lds, bool batch);
// sets sweep_stage / sweep_lds_stage for the coming per-sweep solve
void cd_sweep_mode(cd_ctx* c);
hipError_t cd_launch_decide_batch(hipStream_t stream, const SweepArgs* tab, int B, int jd,
                                  BatchProg* bp);
hipError_t cd_launch_gather_states(hipStream_t stream, const SweepArgs* tab, int B, SolveState* out);
// canonical per-contact friction into slot order (c->mu_slot)
hipError_t cd_launch_mu_scatter(cd_ctx* c, const double* mu);
// adjoint.hip
void cd_adjoint_release(cd_ctx* c);
void cd_window_clear(cd_ctx* c);
int cd_window_begin(cd_ctx* c);      // a new recorded step: starting state
int cd_window_geometry(cd_ctx* c);   // its slot geometry (after preparation)
// frozen-list preparation: geometry, slot constants, warm start, base velocities
hipError_t cd_launch_frozen_refresh(cd_ctx* c);
hipError_t cd_launch_unslot(cd_ctx* c, int final_iter);
int cd_solve_grid(cd_ctx* c);                               // co-resident grid, 0 if none

hipError_t cd_launch_solve(cd_ctx* c, int G, int limit);    // all sweeps in one launch
// update.hip
hipError_t cd_launch_update(cd_ctx* c, int final_iter);
// contacts with R_n > 0 in the canonical forces c->R, into *count (device)
hipError_t cd_launch_count_active(cd_ctx* c, unsigned long long* count);
// velocities of the walls of finite mass after the final forces c->R
// (Eq. 1 for a wall body), into c->d_wall_new (W x dim)
hipError_t cd_launch_wall_velocities(cd_ctx* c);
// per wall of finite mass: its contacts' slots in ascending contact id
hipError_t cd_launch_wall_lists(cd_ctx* c);
hipError_t cd_launch_derived(cd_ctx* c);
SweepArgs cd_sweep_args(cd_ctx* c);

// incidence row width of the sweep's particle gathers
static inline int cd_row_width(int dim) { return dim == 2 ? 8 : 16; }
// doubles the sweep stages per domain particle: V, W, dt/m, dt/I, r, padded
// to an even count (2D: 6, 3D: 10)
__host__ __device__ constexpr int cd_stage_particle(int dim) { return dim == 2 ? 6 : 10; }
// doubles the staged sweep keeps per slot: body pair, normal, g_e/dt, dt w_n,
// dt w_t, previous force, and the friction coefficient when it is per slot
__host__ __device__ constexpr int cd_stage_slot(int dim, bool mu_per_slot) {
  return 1 + (dim == 2 ? 2 : 3) + 3 + dim + (mu_per_slot ? 1 : 0);
}
// doubles per foreign incidence staged for the exchange: the world force F
// and the torque factor (2D: R_t; 3D: n x R)
__host__ __device__ constexpr int cd_stage_halo(int dim) { return dim == 2 ? 3 : 6; }

// slots of the pinned 64-entry scratch (c->h_scratch) that receive the
// sliding and the closed (active) contact counts of a finished solve
constexpr int kSlideSlot = 62;
constexpr int kActiveSlot = 63;
// domains of at most this many particle entries (and workgroups at least
// this wide) stage the foreign incidences' forces in the LDS of their
// particle records (the staged sweep's shared layout)
constexpr int kUnionMax = 128;
// first of the slots (CD_MAX_WALLS * 3 doubles) that receive the velocities
// of the walls after a step with walls of finite mass
constexpr int kWallSlot = 32;

// doubles per slot record.  2D: (R_n, R_t, F_x, F_y).  3D: the frame force
// (R_n, R_t1, R_t2, 0) followed by the contact normal (n_x, n_y, n_z, 0),
// one 64-byte block, so that a reader of a record finds the normal it needs
// in the same cache line; the sweeps rewrite only the force half, both
// record arrays carry the normal.
__host__ __device__ constexpr int cd_rec(int dim) { return dim == 2 ? 4 : 8; }

// 3D tangent basis (t1 = f[3..5], t2 = f[6..8]) of the unit normal f[0..2]:
// the orthonormal basis of Duff et al. (JCGT 6(1), 2017), t1 x t2 = n.  Every
// place that needs the tangents uses these operations, so the values agree.
__device__ inline void cd_tangents(double* f) {
  const double sign = copysign(1.0, f[2]);
  const double aa = -1.0 / (sign + f[2]);
  const double bb = f[0] * f[1] * aa;
  f[3] = 1.0 + sign * f[0] * f[0] * aa;
  f[4] = sign * bb;
  f[5] = -sign * f[0];
  f[6] = bb;
  f[7] = sign + f[1] * f[1] * aa;
  f[8] = -f[1];
}

// 3D: world force F = R_n n + R_t1 t1 + R_t2 t2 and torque factor
// q = R_t1 t2 - R_t2 t1 (n x R) of slot s from its record (force and normal)
__device__ inline void cd_record_force3(const double* rec, int64_t s, double* F, double* Q) {
  const double4 r4 = *(const double4*)(rec + s * cd_rec(3));
  const double4 n4 = *(const double4*)(rec + s * cd_rec(3) + 4);
  double f[9] = {n4.x, n4.y, n4.z, 0, 0, 0, 0, 0, 0};
  cd_tangents(f);
  for (int q = 0; q < 3; ++q) {
    const double fk = r4.x * f[q] + r4.y * f[3 + q];
    F[q] = fk + r4.z * f[6 + q];
    Q[q] = r4.y * f[6 + q] - r4.z * f[3 + q];
  }
}

// helpers
static inline int cd_blocks(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return (int)b;
}
