/* cdhip.h - C ABI of the MI355X (gfx950) Contact Dynamics force solver.
 *
 * The library computes time steps of the non-smooth Contact Dynamics method
 * for rigid frictional disks (2D) and spheres (3D) as described by Shojaaee
 * et al., "An adaptive hierarchical domain decomposition method for parallel
 * contact dynamics simulations of granular materials":
 *   - contact detection with the cell method and a boundary width of
 *     2 vmax dt (Sec. 3.1 and 3.2);
 *   - assignment of contacts to P domains of a hierarchical bisection tree
 *     built for an arbitrary P (Sec. 3.2, Fig. 8), with cuts placed by contact
 *     count (the balancing by contact number named in Sec. 5);
 *   - the iterative force solve: each contact's force is computed with all
 *     other forces fixed (Sec. 2.1, Eqs. 3-9 and Fig. 2); native contacts of a
 *     domain are updated sequentially, other domains' contacts keep the value
 *     of the previous sweep and are exchanged after every sweep (Sec. 3.1);
 *     sweeps stop on the local (I) or global (II) convergence test (Sec. 2.1);
 *   - the semi-implicit Euler update of velocities and positions (Eqs. 1-2).
 *
 * Conventions
 *   - FP64 throughout.  Arrays are structure-of-arrays, component-major:
 *     a[k * n + i].  dim = 2 or 3; dr = 1 (2D) or 3 (3D) rotational components.
 *   - Unless stated otherwise pointers are DEVICE pointers (HIP global memory
 *     on the context's device) owned by the caller; the library copies what it
 *     needs during the call and keeps no caller pointer after it returns.
 *   - Bodies 0..N-1 are particles; a contact partner j >= N is wall j-N.  A
 *     wall is the plane {x : nu.x = o} whose unit normal nu points into the
 *     box.  Contact c joins body 1 = ci[c] < body 2 = cj[c]; its normal n
 *     points from body 1 to body 2 and R is the force on body 2, stored in the
 *     contact frame: (R_n, R_t) in 2D with t = z x n, (R_n, R_t1, R_t2) in 3D.
 *   - All work of a context is enqueued on the stream given at creation.
 *     Calls that return results on the host synchronise that stream.
 *   - Return codes: CD_OK (0); CD_MAXITER (1, a valid but unconverged solve);
 *     negative values are errors, described by cd_last_error().  No C++
 *     exception crosses the ABI.  A context is not thread-safe.
 */
#ifndef CDHIP_H
#define CDHIP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CD_OK = 0,
  CD_MAXITER = 1,        /* sweep cap reached before the convergence test held */
  CD_EINVAL = -1,        /* bad argument (sizes, radii/masses <= 0, skin > 0.2 r_max, P < 1) */
  CD_ENOMEM = -2,        /* device allocation failed */
  CD_ECAPACITY = -3,     /* a domain exceeds the per-domain limits (contacts, colours) */
  CD_ENONFINITE = -4,    /* non-finite input or force */
  CD_EHIP = -5,          /* HIP runtime error; cd_last_error() gives the detail */
  CD_ENOTREADY = -6,     /* particles not set yet */
  CD_ESHADOW = -7        /* the shadow run of a step differed from the first (cd_set_shadow) */
};

/* Solver parameters (host struct, copied at cd_create). */
typedef struct cd_params {
  int dim;               /* 2 or 3 */
  int n_walls;           /* walls are set with cd_set_walls */
  double dt;             /* time step */
  double alpha;          /* convergence threshold on squared relative changes (paper: 1e-6) */
  double mu;             /* Coulomb friction coefficient, all contacts */
  int criterion;         /* 0: local test (I); 1: global test (II) (Sec. 2.1) */
  int max_iter;          /* sweep cap in tolerance mode */
  int fixed_iters;       /* > 0: exactly this many sweeps per step, no convergence stop */
  int overlap_mode;      /* 0: gap clamped at zero in the force law; 1: signed gap */
  int n_domains;         /* P >= 1 domains of the bisection tree */
  int repartition_every; /* rebuild the tree every this many steps (>= 1) */
  int warm_start;        /* 1: start each step from the previous forces of the same pairs */
  double skin;           /* < 0: boundary width 2 vmax dt; >= 0: this fixed width */
} cd_params;

/* Outcome of one step (host struct). */
typedef struct cd_result {
  int status;            /* CD_OK or CD_MAXITER */
  int iterations;        /* sweeps performed */
  int64_t n_contacts;    /* contacts in the list of this step */
  int64_t n_pass;        /* contacts passing the relative test in the last sweep */
  double max_d_fail;     /* largest |dR|^2 among the others (0 if none) */
  double r_avg;          /* mean |R| after the last sweep */
  double r_avg_prev;     /* mean |R| before the last sweep */
  double skin;           /* boundary width used */
  int max_colors;        /* largest number of colours in a domain */
  int max_domain_contacts;  /* largest domain (contacts) */
  int64_t n_active;      /* contacts carrying a force after the solve (R_n > 0) */
  double crit_last;      /* share of contacts passing the relative test (I-a) in the last
                            sweep: n_pass / n_contacts (1 without contacts) */
  double rel_change_last;  /* relative change of the mean force in the last sweep, the
                              quantity of test (II): (dR_avg)^2 / (R_avg + R_avg_prev)^2
                              (0 when both are 0) */
  int64_t n_sliding;     /* closed contacts at the Coulomb bound after the solve, sliding
                            (Eqs. 8-9): 2D |R_t| = mu R_n, 3D |R_t|^2 >= (mu R_n)^2 (1 -
                            1e-12); the other n_active - n_sliding stick, n_contacts -
                            n_active are open */
} cd_result;

/* Time spent in each phase of the last step, milliseconds, from HIP events
 * on the context's stream (host struct). */
typedef struct cd_timing {
  double detect_ms;      /* boundary width, cell binning, pair search, geometry, warm start */
  double partition_ms;   /* tree build or descent */
  double order_ms;       /* per-domain colouring and slot layout */
  double solve_ms;       /* all sweeps, exchange and convergence tests */
  double update_ms;      /* Euler update */
  double sweep_kernel_ms;  /* duration of the solve kernel (one-launch mode), or the
                            mean duration of the timed sweep launches times the sweeps
                            executed (per-sweep mode) */
  int sweep_launches;    /* solve / sweep kernel launches in the last step */
  int sweeps_executed;   /* sweeps computed, including the one the stop decision overlaps */
  int block_threads;     /* threads of the workgroup that sweeps one domain */
  int sweeps_timed;      /* sweep launches inside the timed groups (per-sweep mode) */
  int staged;            /* 1: the sweeps read each domain's contact data from LDS;
                            2: and workgroup 0 also took each stop decision */
  int global_records;    /* 1: a domain's particle records did not fit in LDS and the
                            sweeps kept them in global memory */
  int foreign_in_lds;    /* 1: with staged contact data, the previous sweep's forces of
                            each domain's foreign incidences were staged in LDS as well,
                            so that the exchange read no record from memory (Sec. 3.1) */
} cd_timing;

typedef struct cd_ctx cd_ctx;

/* Create a context for n_particles bodies (Sec. 2.1: rigid disks or spheres,
 * each with mass, moment of inertia and radius) on the current HIP device.
 * contact_capacity > 0 sizes the contact arrays for that many contacts up
 * front, so that steps with at most that many contacts do not reallocate
 * them; 0 sizes them at the first step.  Either way they grow by a quarter when a
 * step needs more.  stream: a hipStream_t (NULL = the null stream) on which
 * all work runs.  The context owns its workspace and frees it in cd_destroy.
 * CD_EINVAL for dim not 2 or 3, N < 1, P < 1, dt <= 0, more than 8 walls or
 * a negative capacity; CD_ENOMEM when the workspace does not fit. */
int cd_create(cd_ctx** out, const cd_params* params, int64_t n_particles,
              int64_t contact_capacity, void* stream);
int cd_destroy(cd_ctx* ctx);

/* Particle state and properties (Sec. 2.1, Eqs. 1-2; device pointers,
 * copied in): x, v (dim x N); w (dr x N, NULL = 0); radius, mass, inertia
 * (N), all positive and finite, else CD_EINVAL.  Starts a new simulation:
 * the step counter, the tree and the warm-start list are reset. */
int cd_set_particles(cd_ctx* ctx, const double* x, const double* v, const double* w,
                     const double* radius, const double* mass, const double* inertia);

/* External forces (dim x N) and torques (dr x N), the F_i of Eq. (1) and
 * its rotational analogue; device pointers, NULL = zero. */
int cd_set_external(cd_ctx* ctx, const double* force, const double* torque);

/* Walls, bodies of prescribed motion (Sec. 2.1), HOST pointers: normal
 * (W x dim, unit, into the box), offset (W), velocity (W x dim, NULL = at
 * rest).  W must equal params.n_walls. */
int cd_set_walls(cd_ctx* ctx, const double* normal, const double* offset, const double* velocity);

/* Simulation box (HOST pointers, dim each): the root region of the
 * bisection tree (Sec. 3.2, Fig. 8) and the extent of the cell grid
 * (Sec. 3.2).  Box faces lying on an axis-aligned wall move with that wall.
 * CD_EINVAL unless hi > lo on every axis. */
int cd_set_box(cd_ctx* ctx, const double* lo, const double* hi);

/* Boundary conditions of the paper's benchmark setups (Sec. 4.1, Fig. 10:
 * periodic in x between confining walls under pressure; Sec. 4.4: the same
 * walls sliding in opposite directions), from the next step on.
 *   periodic_mask: bit k makes axis k periodic with the box's length
 *     (cd_set_box): particle pairs are taken at their nearest image, the
 *     cell grid wraps (at least three cells of 2.2 r_max along the axis,
 *     else the step returns CD_EINVAL), positions and contact positions are
 *     kept in [lo, hi).  No wall may bound a periodic axis (CD_EINVAL).
 *   wall_inv_mass (HOST, W, NULL = all 0): 1/M of each wall; a wall with
 *     1/M > 0 is a body of the solve that moves along its normal only: its
 *     contacts conflict in the colouring (distinct colours), each domain
 *     touching it keeps its own copy of its velocity, recomputed in every
 *     exchange as u_n + dt/M (F - sum of R_n over all its contacts, ascending
 *     contact id) along its normal (Eq. 1 for the wall), its tangential
 *     velocity (cd_set_walls) stays prescribed, and after the step it keeps
 *     the velocity of the final forces.  1/M = 0: prescribed motion.
 *   wall_force (HOST, W, NULL = all 0): the constant external force F on
 *     each wall along its normal (pressure times area).
 * Walls of finite mass exclude the mixed update, the random order, load
 * measurement, the one-launch solve (mode 0), the batch and the adjoint
 * (CD_EINVAL where they are set); periodic axes exclude the adjoint. */
int cd_set_boundary(cd_ctx* ctx, int periodic_mask, const double* wall_inv_mass,
                    const double* wall_force);

/* One time step: detection, warm start, partition, order, force solve,
 * Euler update (Fig. 7).  Positions and velocities are updated in place in
 * the context.  out (host, may be NULL) receives the outcome.  Returns
 * CD_OK, CD_MAXITER or an error. */
int cd_step(cd_ctx* ctx, cd_result* out);

/* The iterative force solve alone (Sec. 2.1 sweeps and tests, Sec. 3.1
 * domain-wise update and exchange) on a contact list the caller gives, at
 * the context's current positions, velocities and walls; no detection and
 * no time step.  All pointers are DEVICE pointers of n_c entries:
 *   ci, cj   the list in canonical order: 0 <= ci < N, ci < cj < N + W, the
 *            keys (ci, cj) strictly increasing (the order of cd_get_contacts);
 *   dom      the domain of each contact, in [0, P); NULL: the contact-count
 *            bisection of the mid-gap positions (Sec. 3.2, Fig. 8);
 *   order    the sequential update order: the contacts of domain 0, then
 *            of domain 1, ..., each domain's in the order they are to be
 *            updated (a permutation of 0..n_c-1 with non-decreasing
 *            dom[order[s]]; needs dom); NULL: first-fit colour-major order.
 *            A given order is run colour by colour with colour = one above
 *            the highest colour of the earlier contacts sharing a body, which
 *            is the same sequential order; CD_ECAPACITY when it needs more
 *            than 64 colours in a domain;
 *   R_inout  (dim x n_c, contact frame) the starting forces, overwritten
 *            with the forces after the last sweep.
 * The normals, gaps and constants follow from the context's positions
 * (Fig. 1, Eq. 5).  The list and its forces become the context's current
 * list: cd_get_contacts returns them and the next cd_step warm-starts from
 * them.  out (host, may be NULL) receives the outcome (skin = 0).  Returns
 * CD_OK, CD_MAXITER or an error: CD_EINVAL when the list, dom or order
 * fails its checks (nothing is solved), for an order without dom or
 * together with the mixed update or the random order, and while the
 * adjoint records (cd_set_adjoint); CD_ENOTREADY before cd_set_particles /
 * cd_set_box. */
int cd_solve_contacts(cd_ctx* ctx, int64_t n_c, const int32_t* ci, const int32_t* cj,
                      const int32_t* dom, const int32_t* order, double* R_inout,
                      cd_result* out);

/* Copy the state after the steps so far out (Eqs. 1-2; device pointers,
 * NULL skips): x, v (dim x N), w (dr x N). */
int cd_get_state(cd_ctx* ctx, double* x, double* v, double* w);

/* Wall offsets after the steps so far (HOST pointer, W entries): each wall
 * has moved by dt times its normal velocity per step (Sec. 2.1). */
int cd_get_walls(cd_ctx* ctx, double* offset);

/* Wall velocities after the steps so far (HOST pointer, W x dim): as set,
 * with the normal part of walls of finite mass evolved (cd_set_boundary). */
int cd_get_wall_velocities(cd_ctx* ctx, double* velocity);

/* Number of contacts in the context's current list (Sec. 3.1: pairs within
 * the boundary width; host value, no device work). */
int64_t cd_num_contacts(const cd_ctx* ctx);

/* The contacts of the last step in canonical (ci, cj) order (device
 * pointers, NULL skips): ci, cj (nc), normal (dim x nc) and gap (nc) of
 * Fig. 1, R (dim x nc, contact frame, Eqs. 3-9), dom (nc, the domain of the
 * contact's mid-gap position, Sec. 3.1), color (nc) and slot_contact (nc:
 * the contact at each position of the domain-major sequential update
 * order).  cap must be >= cd_num_contacts(), else CD_EINVAL. */
int cd_get_contacts(cd_ctx* ctx, int64_t cap, int32_t* ci, int32_t* cj, double* normal,
                    double* gap, double* R, int32_t* dom, int32_t* color,
                    int32_t* slot_contact);

/* The current bisection tree, 2P-1 nodes in creation order (HOST pointers):
 * axis (-1 for leaves), cut, child (2 per node, -1 for leaves), leaf domain
 * id (-1 for inner nodes). */
int cd_get_tree(cd_ctx* ctx, int32_t* axis, double* cut, int32_t* child, int32_t* leaf);

/* Snapshots for checkpoint and resume.  A time step depends on the
 * positions and velocities (Eq. 1), the walls' offsets and velocities, the
 * step counter (tree rebuilds every repartition_every steps, Sec. 3.2; the
 * random order's draws), the previous step's contact list and forces (the
 * warm start) and the bisection tree the tree descent reuses (Sec. 3.2),
 * plus the load-balancing capacities (Sec. 3.3) when set.  A snapshot holds
 * exactly that, so that a context loaded from it steps bitwise as the one it
 * was taken from would have.
 *
 * cd_snapshot_size: the bytes of a snapshot of the current state (host
 * value).  cd_snapshot_save: writes it into the caller's HOST buffer of
 * that many bytes (CD_EINVAL for another size).  cd_snapshot_load: restores
 * one into a context created with the same parameters, particle count,
 * walls and domain count, whose particles (radii, masses, inertia), box,
 * boundary conditions and other settings the caller has set as in the
 * original (the snapshot overwrites x, v, w, the walls' offsets and
 * velocities, the box faces that follow walls, the step counter, the
 * contact list and forces, the tree and the capacities; until the next
 * step, cd_get_contacts returns CD_ENOTREADY, the contacts' geometry,
 * domains and colours being rebuilt by that step).  Both run between
 * steps only (CD_ENOTREADY after cd_prepare) and are refused with a kept
 * contact list or the adjoint on (CD_EINVAL); a buffer that is not a
 * snapshot of a matching context (header, size, split axes) is refused with
 * CD_EINVAL before anything changes. */
int cd_snapshot_size(cd_ctx* ctx, int64_t* bytes);
int cd_snapshot_save(cd_ctx* ctx, void* buf, int64_t bytes);
int cd_snapshot_load(cd_ctx* ctx, const void* buf, int64_t bytes);

/* Shadow mode, a check for nondeterminism (debugging; each step costs about
 * twice as much).  mode 1: every cd_step takes a snapshot, steps, keeps the
 * results (positions, velocities, contact list, forces, walls, sweep count
 * and status), loads the snapshot, steps again and compares the two runs
 * bitwise; a difference returns CD_ESHADOW with the first differing
 * quantity in cd_last_error, else the second run's result.  The
 * domain-wise solve is deterministic by construction (fixed-order
 * reductions, no floating-point atomics), so any difference is a fault.
 * mode 2 is the mode's own self-test: the second run starts with the first
 * velocity component 1e-9 away from the snapshot's, which must be reported
 * (the step's result is then the second run's).  mode 0 (the
 * default) steps once.  Refused (CD_EINVAL) with a kept contact list or the
 * adjoint on; cd_prepare / cd_solve and the batch step once regardless. */
int cd_set_shadow(cd_ctx* ctx, int mode);

/* every > 0: split sweep launches 2, 3, ... into consecutive groups of
 * `every` and bracket each group with one pair of HIP events;
 * cd_timing.sweep_kernel_ms is the mean launch duration over the complete
 * groups of working launches times the sweeps executed.  0 records no
 * per-sweep events.  Default 1 (every launch on its own). */
int cd_set_timing(cd_ctx* ctx, int every);

/* mode 1 (default): one launch per sweep; an extra workgroup of each launch
 * takes the stop decision of the previous sweep, so the launch after the
 * stopping sweep computes a sweep whose result is discarded.  Each domain's
 * contact data is copied to LDS alongside the exchange when that keeps every
 * workgroup of a launch resident at once; otherwise each thread reads its
 * contact of the next colour into registers one colour ahead.
 * mode 2: as mode 1, always in the register form.
 * mode 0: all sweeps of a step in one launch, blocks synchronised by a grid
 * barrier, the stop decision overlapping the next sweep.  Same results in
 * every mode. */
int cd_set_solve_mode(cd_ctx* ctx, int mode);

/* Threads of the workgroup that sweeps one domain: 64, 128, 192 or 256;
 * 0 (default) picks 128, or 64 when no domain has more than 64 contacts
 * and 64 particles; -1 tunes it: the next four steps run with 64, 128, 192
 * and 256 threads (results do not depend on the width), the width with the
 * fastest mean sweep launch is kept, and the choice is cached for the
 * process per (dimension, log2 N, log2 P, device) so that later contexts of
 * the same kind start with it.  Tuning needs sweep timing (cd_set_timing
 * with every > 0). */
int cd_set_launch(cd_ctx* ctx, int block_threads);

/* Mixed sequential/parallel update (Sec. 2.3) from the next step on: the
 * contacts whose pair number u(seed, i, j) in [0, 1) - the top 53 bits of
 * SplitMix64(SplitMix64(SplitMix64(seed) ^ i) ^ j) - falls below p are
 * updated in parallel: each takes its new force from the velocities at the
 * start of the sweep (all other forces at their previous values) and its
 * change reaches the other contacts only through the next exchange; the
 * rest are updated sequentially as before.  Such contacts form colour 0 of
 * their domain (cd_get_contacts), the sequential ones colour from 1.  p >= 1
 * updates every contact in parallel (the Jacobi scheme); p < 0 (default)
 * none.  CD_EINVAL for p = NaN or together with the adjoint. */
int cd_set_mixed_update(cd_ctx* ctx, double p, unsigned long long seed);

/* Random sequential order (Sec. 2.1) from the next step on (on != 0): in
 * every sweep each domain updates its own contacts one at a time in a
 * random order drawn afresh for that sweep, instead of colour by colour.
 * Slot s (the contact's position in the domain-major, colour-major slot
 * order of cd_get_contacts) draws SplitMix64(SplitMix64(K ^ j) ^ s) in
 * sweep j (1-based) of time step t, K = SplitMix64(SplitMix64(seed) ^ t), t
 * the number of steps the context has taken; a domain takes its slots by
 * increasing draw, equal draws by slot.  The domain semantics (frozen
 * foreign contacts, exchange between sweeps) are unchanged.  One thread per
 * domain runs the updates, so a sweep is much slower than the colour-major
 * one: the mode is for comparing orders (Sec. 4.3), not for throughput.
 * Needs 16 bytes of LDS per contact of the largest domain: the step's
 * preparation keeps the particle records in global memory when they do not
 * fit beside them, and the solve returns CD_ECAPACITY when the draws alone
 * do not fit (or when the mode was switched on after cd_prepare, whose
 * sizing did not include them).  CD_EINVAL
 * together with the mixed update, the adjoint or load measurement; the
 * one-launch solve (mode 0) and the batch refuse it.  on = 0: colour-major
 * (default). */
int cd_set_random_order(cd_ctx* ctx, int on, unsigned long long seed);

/* Adaptive load balancing (Sec. 3.3).  sigma_star >= 0 switches load
 * measurement on: every sweep launch records, per domain, the real time its
 * workgroup spends on it (per-sweep launches only: solve modes 1 and 2, not the
 * one-launch mode 0, not batched sweeps), summed over the step.  After each
 * step the imbalance sigma_T = sqrt(<T^2> - <T>^2) / <T> over the P domain
 * times T_i is computed; when sigma_T >= sigma_star the per-domain
 * capacities become n_i / T_i (n_i the domain's contacts in that step), and
 * every later tree rebuild (cd_params.repartition_every) cuts each inner
 * node so that its left branch receives the share nu_L / (nu_L + nu_R) of
 * the node's contacts, nu of a branch summing the capacities of its leaves
 * (a domain without contacts or time counts as the mean capacity).  Below
 * the threshold the last capacities stay in force, as the paper keeps the
 * domain configuration.  sigma_star < 0 (default) switches measurement off
 * and returns to leaf-count cuts.  CD_EINVAL for a non-finite threshold,
 * CD_ENOMEM / CD_EHIP when the measurement buffers or the clock rate are
 * unavailable. */
int cd_set_load_balance(cd_ctx* ctx, double sigma_star);

/* Capacities for the tree rebuilds from now on (host array of P doubles in
 * domain order, copied), in place of measured ones: for tests and for
 * callers with a cost model of their own.  NULL returns to leaf-count
 * cuts.  Measured capacities (cd_set_load_balance) replace them when the
 * threshold is reached. */
int cd_set_domain_capacity(cd_ctx* ctx, const double* capacity);

/* The last measured step's per-domain times in microseconds (host array of
 * P doubles, or NULL) and their sigma_T (or NULL).  CD_ENOTREADY before a
 * measured step. */
int cd_get_domain_times(cd_ctx* ctx, double* times_us, double* sigma_t);

/* Phase timings of the last step (host struct), the phases of Fig. 7. */
int cd_get_timing(cd_ctx* ctx, cd_timing* out);

/* Static description of a status code, and the last error of a context
 * (plumbing: no passage of the paper defines them). */
const char* cd_status_string(int status);
const char* cd_last_error(const cd_ctx* ctx);

/* ---- A step in phases, per-contact friction, adjoint ---------------------
 * cd_step = cd_prepare + cd_solve.  Between the two the contact list of the
 * coming solve is known (cd_num_contacts, cd_get_contacts), so per-contact
 * inputs can be given in its canonical order. */

/* Boundary width, detection, warm start, partition and order of the coming
 * step (the first part of cd_step). */
int cd_prepare(cd_ctx* ctx);

/* Friction coefficient of every contact of the prepared list (DEVICE array
 * of cd_num_contacts doubles, canonical order), for the coming cd_solve only
 * (Sec. 2.1 allows a coefficient per contact).  CD_ENOTREADY without
 * cd_prepare. */
int cd_set_contact_mu(cd_ctx* ctx, const double* mu);

/* The solve and the Euler update of the prepared step (the rest of cd_step). */
int cd_solve(cd_ctx* ctx, cd_result* out);

/* checkpoint_every > 0: solves with a fixed sweep count (params.fixed_iters)
 * record the forces before the first sweep and after every checkpoint_every
 * sweeps, for cd_adjoint (2D).  0 (default): no recording.  CD_EINVAL for
 * checkpoint_every > 0 on a 3D context, with walls of finite mass or periodic
 * axes, the mixed update or the random order. */
int cd_set_adjoint(cd_ctx* ctx, int checkpoint_every);

/* on != 0 (2D): the next step detects, partitions and orders as usual and
 * every later step keeps that contact list, tree and colouring: it only
 * recomputes normals and gaps at the new positions (Sec. 2.1, Fig. 1),
 * starts from the previous step's forces and solves.  Contacts that would
 * form meanwhile are not seen, so keep the window short against the skin.
 * Per-contact friction set with cd_set_contact_mu stays in force over the
 * kept steps.  With cd_set_adjoint active, all steps since the list was
 * built form the window that cd_adjoint reverses (without a kept list the
 * window is the last step).  on = 0 returns to per-step detection; a new
 * cd_set_particles also rebuilds the list.  CD_EINVAL in 3D. */
int cd_set_frozen_list(cd_ctx* ctx, int on);

/* Reverse mode of the recorded window (the last step, or every step since
 * the kept list was built, see cd_set_frozen_list): given dL_dR (DEVICE,
 * dim x n_c, canonical order, frame components (R_n, R_t) of the forces
 * after the last sweep of the last step), writes dL_dmu (DEVICE, n_c: per
 * contact friction, summed over the window's steps), dL_dv (DEVICE, dim x N)
 * and dL_dw (DEVICE, N) of the velocities the window's first step started
 * from; any output may be NULL.  Over several steps the chain runs through
 * each step's velocity and position update (Eqs. 1-2) and its normals and
 * gaps; the forces the first step started from count as constants.  The sweeps are differentiated exactly in the
 * branch each contact took (open, stick, slide; Eqs. 3-9), segment by
 * segment from the checkpoints.  The slot data of the solve must still be in
 * place: call it before the next cd_prepare / cd_step.  CD_ENOTREADY without
 * a recorded solve, CD_EINVAL in 3D, CD_ECAPACITY when a domain is too large
 * for the reverse sweep's LDS.  Motivation: gradients of contact forces with
 * respect to friction and initial velocities for inverse problems and
 * calibration, on top of the paper's fixed-iteration option (Sec. 2.1). */
int cd_adjoint(cd_ctx* ctx, const double* dL_dR, double* dL_dmu, double* dL_dv, double* dL_dw);

/* cd_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same reverse pass with the same results, bit for bit, but its workspace
 * (the adjoints of forces, velocities and positions, the recomputed
 * segment's forces, the particle-to-entry lists, the recomputing sweeps'
 * state) is carved out of one static array of 64 MiB per device that the
 * library holds from its load until the process ends; the call makes no
 * hipMalloc or hipFree and clears what must start at zero with kernels.
 * Every call on a device shares that device's array and leaves its
 * contents behind: calls that overlap on one device (two threads, two
 * streams) race and must be serialised by the caller.  The workspace
 * needs (16 cap + 4 C cap) doubles + 2 cap ints per contact slot of
 * capacity cap (C = checkpoint interval) plus 15 doubles + 2 ints per
 * particle; CD_ECAPACITY when that exceeds 64 MiB (outputs untouched), and
 * also when the context's prefix-scan workspace was not sized by a
 * prepared step.  Other errors as cd_adjoint. */
int cd_adjoint_static(cd_ctx* ctx, const double* dL_dR, double* dL_dmu, double* dL_dv,
                      double* dL_dw);

/* ---- Batches of independent packings ------------------------------------
 * Many packings stepped together: each packing is a context created and
 * filled as above (its own parameters, friction, domain count, walls); the
 * batch runs, per time step, every packing's detection, partition and order,
 * then ONE kernel launch per sweep over the domains of all packings whose
 * solve is still open (per-packing stop decisions; stopped packings idle),
 * then every packing's update.  A packing's results equal those of cd_step
 * on that context alone: same list, partition, order and arithmetic.
 * Motivation: the paper's one-process-per-domain scheme (Sec. 3) applied to
 * many small systems at once keeps a GPU full where one small packing
 * cannot. */
typedef struct cd_batch cd_batch;

typedef struct cd_batch_timing {
  double prepare_ms;       /* detection, partition and order of all packings */
  double solve_ms;         /* the batched sweeps and decisions */
  double finish_ms;        /* canonical forces and updates of all packings */
  double sweep_kernel_ms;  /* mean timed sweep launch x sweeps executed */
  int sweep_launches;      /* batched sweep launches */
  int sweeps_executed;     /* launches that did work for some packing */
  int sweeps_timed;        /* launches inside the timed groups */
  int block_threads;       /* threads per domain workgroup */
  int workgroups;          /* workgroups of one batched launch */
  int staged;              /* 1: the sweeps read each domain's contact data from LDS */
} cd_batch_timing;

/* ctxs: `count` contexts (host array of handles), all of one dimension, on
 * one device and one stream; the batch keeps the handles (the caller keeps
 * ownership and must not destroy a context while the batch lives) and uses
 * their stream.  While it belongs to a batch a context records no events
 * around its phases (cd_get_timing's phase times read 0; the batch times
 * its phases in cd_batch_timing).  CD_EINVAL for mismatched contexts. */
int cd_batch_create(cd_batch** out, cd_ctx* const* ctxs, int count);
int cd_batch_destroy(cd_batch* batch);

/* Per-sweep event timing of the batched launches, as cd_set_timing. */
int cd_batch_set_timing(cd_batch* batch, int every);

/* One time step of every packing.  results: host array of `count`
 * cd_result, filled for every packing.  A packing whose solve diverges
 * (non-finite force, or velocities beyond the displacement bound at the next
 * step: the instability of the mixed parallel/sequential update, Sec. 2.3)
 * leaves the batch: its result status is CD_ENONFINITE or CD_EINVAL from then
 * on and the others go on.  Returns CD_OK, CD_MAXITER (some packing hit its
 * sweep cap), CD_ENONFINITE (some packing has left the batch), or the error
 * of the first packing whose preparation failed otherwise (named by
 * cd_batch_last_error); CD_ECAPACITY when a packing's domain does not fit in
 * LDS (use more domains for it). */
int cd_batch_step(cd_batch* batch, cd_result* results);
int cd_batch_get_timing(cd_batch* batch, cd_batch_timing* out);
const char* cd_batch_last_error(const cd_batch* batch);

#ifdef __cplusplus
}
#endif
#endif
