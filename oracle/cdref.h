/* cdref.h - FP64 CPU oracle of the Contact Dynamics contact-force solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library and must never be used as a
 * fallback for it.
 *
 * What it computes (Shojaaee et al., "An adaptive hierarchical domain
 * decomposition method for parallel contact dynamics simulations of granular
 * materials"):
 *   - the first-order semi-implicit Euler step, Sec. 2.1, Eqs. (1)-(2);
 *   - the single-contact force law (velocity-Signorini plus Coulomb cone),
 *     Sec. 2.1, Eqs. (3)-(9) and Fig. 2;
 *   - the iterative sequential (nonlinear Gauss-Seidel) sweep and the local
 *     (I) and global (II) convergence tests, Sec. 2.1;
 *   - the domain-wise sweep: native contacts updated sequentially, foreign
 *     contacts frozen at the previous sweep's value, Sec. 3.1;
 *   - cell-method contact detection with boundary width 2 vmax dt, Sec. 3.1-3.2;
 *   - the hierarchical (orthogonal recursive bisection) domain tree for an
 *     arbitrary processor count, Sec. 3.2 and Fig. 8, with cuts placed by
 *     contact count (the "most exact" balancing named in Sec. 5).
 *
 * Conventions shared by every function:
 *   - arrays are structure-of-arrays, component-major: a[k*n + i];
 *   - bodies 0..N-1 are particles; a contact partner j >= N is wall j-N;
 *   - a wall is the plane {x : nu.x = o} with unit normal nu into the box;
 *   - contact c = (ci[c], cj[c]) with ci < cj; body 1 = ci, body 2 = cj;
 *     the normal n points from body 1 to body 2; R is the force on body 2;
 *   - contact forces are stored in the contact frame: (R_n, R_t) in 2D and
 *     (R_n, R_t1, R_t2) in 3D, component-major with stride n_contacts.
 */
#ifndef CDREF_H
#define CDREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CDREF_OK = 0,
  CDREF_MAXITER = 1,
  CDREF_EINVAL = -1,
  CDREF_ENOMEM = -2,
  CDREF_ECAPACITY = -3,
  CDREF_ENONFINITE = -4
};

typedef struct {
  int dim;             /* 2 or 3 */
  int n_walls;
  double dt;
  double alpha;        /* convergence threshold (paper: 1e-6) */
  double mu;           /* friction coefficient when no per-contact values */
  int criterion;       /* 0: local test (I); 1: global test (II) */
  int max_iter;        /* sweep cap in tolerance mode */
  int fixed_iters;     /* > 0: exactly this many sweeps */
  int overlap_mode;    /* 0: gap clamped at 0 (g_e = max(g,0)); 1: signed gap */
  int n_domains;       /* P >= 1 */
  int repartition_every; /* rebuild the tree every this many steps (>= 1) */
  int warm_start;      /* 1: start each step from the previous step's forces */
  double skin;         /* < 0: 2 vmax dt */
} cdref_params;

#define CDREF_MAX_WALLS 8

/* Walls whose motion along their normal follows from the contact forces: a
 * wall of finite mass M under a constant external force F along its normal
 * nu (the pressure-controlled confining walls of Sec. 4.1); its velocity
 * along the wall stays prescribed (the shearing walls of Sec. 4.4).  In the
 * solve such a wall is a body like a particle: each domain keeps its own
 * copy of its velocity, updated by the domain's contacts with it, and the
 * exchange recomputes it from all its contact forces of the previous sweep.
 * inv_mass[w] = 0: the wall's motion is prescribed. */
typedef struct {
  const double* normal;     /* W x dim, unit, into the box */
  const double* inv_mass;   /* W: 1/M */
  const double* force;      /* W: F along nu */
} cdref_mobile_walls;

typedef struct {
  int status;
  int iterations;
  int64_t n_contacts;
  /* criterion values of the last evaluated sweep */
  int64_t n_pass;          /* contacts passing the relative test */
  double max_d_fail;       /* max |dR|^2 over contacts failing it (0 if none) */
  double r_avg;            /* mean |R| after the last sweep */
  double r_avg_prev;       /* mean |R| before the last sweep */
  double skin;
} cdref_info;

/* Candidate contacts: particle pairs and particle-wall pairs whose gap is
 * <= skin (Sec. 3.1, boundary width).  Output in canonical (i, j) order.
 * use_cells = 0: brute force O(N^2); 1: cell method over [box_lo, box_hi]
 * with mesh >= 2.2 r_max (Sec. 3.2).  Returns CDREF_ECAPACITY with *nc set
 * to the required size when cap is too small. */
int cdref_detect(int dim, int64_t n, const double* x, const double* r,
                 int n_walls, const double* wall_normal, const double* wall_offset,
                 double skin, int use_cells, const double* box_lo, const double* box_hi,
                 int64_t cap, int32_t* ci, int32_t* cj, int64_t* nc);

/* cdref_detect in a box with periodic axes (the benchmark boxes of Sec. 4.1
 * are periodic in x): period[k] > 0 is the length of axis k, which must
 * equal box_hi[k] - box_lo[k]; particle pairs are taken at their nearest
 * image and the cells wrap around (at least three along a periodic axis,
 * else CDREF_EINVAL).  period = NULL: as cdref_detect. */
int cdref_detect_bc(int dim, int64_t n, const double* x, const double* r,
                    int n_walls, const double* wall_normal, const double* wall_offset,
                    double skin, int use_cells, const double* box_lo, const double* box_hi,
                    const double* period, int64_t cap, int32_t* ci, int32_t* cj, int64_t* nc);

/* Per-contact geometry (Sec. 2.1, Fig. 1): unit normal n (dim x nc), gap g
 * and the contact position at the middle of the gap (Sec. 3.1). */
void cdref_geometry(int dim, int64_t n, const double* x, const double* r,
                    int n_walls, const double* wall_normal, const double* wall_offset,
                    int64_t nc, const int32_t* ci, const int32_t* cj,
                    double* normal, double* gap, double* xmid);

/* cdref_geometry with periodic axes: the nearest image of each particle
 * pair, the contact position taken back into [box_lo, box_lo + period). */
void cdref_geometry_bc(int dim, int64_t n, const double* x, const double* r,
                       int n_walls, const double* wall_normal, const double* wall_offset,
                       const double* period, const double* box_lo, int64_t nc,
                       const int32_t* ci, const int32_t* cj, double* normal, double* gap,
                       double* xmid);

/* Hierarchical bisection tree for P leaves (Sec. 3.2, Fig. 8), cuts placed
 * by contact count.  Node arrays have 2P-1 entries in creation order:
 * axis and cut of inner nodes, children (2 per node, -1 for leaves), leaf
 * domain id (-1 for inner nodes), and the leaf count below each node.
 * dom[c] receives the leaf (domain) of each contact. */
int cdref_orb(int dim, int P, const double* box_lo, const double* box_hi,
              int64_t nc, const double* xmid,
              int32_t* node_axis, double* node_cut, int32_t* node_child,
              int32_t* node_leaf, int32_t* node_leaves, int32_t* dom);

/* The same with the cuts placed by capacity (Sec. 3.3): the left branch of
 * every inner node receives the share nu_L / (nu_L + nu_R) of the node's
 * contacts (k = floor(n share), at most n - 1), nu of a branch summing the
 * capacities (P doubles, domain order) of its leaves; NULL capacity: leaf
 * counts, as cdref_orb. */
int cdref_orb_capacity(int dim, int P, const double* box_lo, const double* box_hi,
                       int64_t nc, const double* xmid, const double* capacity,
                       int32_t* node_axis, double* node_cut, int32_t* node_child,
                       int32_t* node_leaf, int32_t* node_leaves, int32_t* dom);

/* The left-branch shares of the inner nodes for P capacities (2P-1 entries,
 * 0 for leaves); capacities that are not positive and finite count as the
 * mean of the valid ones (1 if none). */
int cdref_balance_fractions(int P, const double* capacity, double* node_frac);

/* Mixed sequential/parallel update (Sec. 2.3).  The pair number
 * u(seed, i, j) in [0, 1): top 53 bits of SplitMix64(SplitMix64(SplitMix64(seed)
 * ^ i) ^ j); a contact is updated in parallel when u < p. */
double cdref_pair_uniform(uint64_t seed, int64_t i, int64_t j);
void cdref_parallel_flags(int64_t nc, const int32_t* ci, const int32_t* cj, double p,
                          uint64_t seed, uint8_t* flags);
/* order with parallel contacts (flags, or NULL): they take colour 0 and come
 * first in their domain; the others are coloured first-fit from colour 1 */
int cdref_order_mixed(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj,
                      int P, const int32_t* dom, const uint8_t* parallel, int32_t* color,
                      int32_t* slot_contact, int64_t* dom_start);
/* solve in which each domain first computes its parallel contacts from the
 * velocities of the exchange without applying their changes, then updates
 * the others sequentially */
int cdref_solve_mixed(const cdref_params* p, int64_t n, const double* v, const double* w,
                      const double* r, const double* m, const double* inertia,
                      const double* f, const double* t, const double* wall_velocity,
                      int64_t nc, const int32_t* ci, const int32_t* cj,
                      const double* normal, const double* gap, const double* mu_c,
                      const uint8_t* parallel, int P, const int64_t* dom_start,
                      const int32_t* slot_contact, double* R, cdref_info* info,
                      double* history);

/* Random sequential order (Sec. 2.1): in sweep j (1-based) of time step
 * `step` each domain updates its contacts one at a time in the order of
 * increasing draw SplitMix64(SplitMix64(K ^ j) ^ s), s the slot, equal draws
 * by slot, K = SplitMix64(SplitMix64(seed) ^ step). */
/* Threads over which the domains of each sweep are spread (OpenMP; 1, the
 * default, runs them one after another).  The domains of a sweep are
 * independent, so the results do not depend on it. */
void cdref_set_threads(int threads);
uint64_t cdref_random_step_key(uint64_t seed, int64_t step);
uint64_t cdref_random_slot_key(uint64_t step_key, int j, int64_t s);
int cdref_solve_random(const cdref_params* p, int64_t n, const double* v, const double* w,
                       const double* r, const double* m, const double* inertia,
                       const double* f, const double* t, const double* wall_velocity,
                       int64_t nc, const int32_t* ci, const int32_t* cj,
                       const double* normal, const double* gap, const double* mu_c, int P,
                       const int64_t* dom_start, const int32_t* slot_contact, uint64_t seed,
                       int64_t step, double* R, cdref_info* info, double* history);

/* The solve with walls of finite mass (mw, NULL: all prescribed) and the
 * mixed update's parallel flags (NULL: none); otherwise as cdref_solve. */
int cdref_solve_bc(const cdref_params* p, int64_t n, const double* v, const double* w,
                   const double* r, const double* m, const double* inertia,
                   const double* f, const double* t, const double* wall_velocity,
                   int64_t nc, const int32_t* ci, const int32_t* cj,
                   const double* normal, const double* gap, const double* mu_c,
                   const uint8_t* parallel, int P, const int64_t* dom_start,
                   const int32_t* slot_contact, const cdref_mobile_walls* mw, double* R,
                   cdref_info* info, double* history);

/* Wall velocities after forces R (Eq. 1 for the wall bodies): a wall of
 * finite mass takes u_n + dt/M (F - sum of its contacts' R_n, ascending
 * contact id) along its normal and keeps its tangential velocity; the
 * others keep theirs.  U: W x dim. */
void cdref_wall_velocities(int dim, int64_t n, double dt, int W, const double* wall_velocity,
                           const cdref_mobile_walls* mw, int64_t nc, const int32_t* cj,
                           const double* R, double* U);

/* Load imbalance sigma_T = sqrt(<T^2> - <T>^2) / <T> over P times (Sec. 3.3). */
double cdref_sigma_t(int P, const double* T);

/* Assign contacts to domains by descending an existing tree (Sec. 3.2). */
void cdref_descend(int dim, int P, const int32_t* node_axis, const double* node_cut,
                   const int32_t* node_child, const int32_t* node_leaf,
                   int64_t nc, const double* xmid, int32_t* dom);

/* Leaf counts of the paper's tree shape for P leaves (Fig. 8); out has
 * 2P-1 entries in creation order.  Exposed for tests. */
int cdref_tree_leaves(int P, int32_t* node_leaves);

/* cdref_order_mixed where the walls in mobile_mask (bit w: wall w has
 * finite mass) conflict like particles: their contacts take distinct
 * colours, since each changes the wall's velocity. */
int cdref_order_bc(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj, int P,
                   const int32_t* dom, const uint8_t* parallel, int mobile_mask, int32_t* color,
                   int32_t* slot_contact, int64_t* dom_start);

/* Update order inside each domain: greedy first-fit colouring of the
 * domain's contacts in canonical order (two contacts conflict when they
 * share a particle; walls never conflict), then order by (colour, id).
 * Outputs color[c], slot_contact[s] (domain-major order) and dom_start[P+1]. */
int cdref_order(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj,
                int P, const int32_t* dom, int32_t* color, int32_t* slot_contact,
                int64_t* dom_start);

/* The iterative force solve of one time step (Sec. 2.1 and 3.1).  Particle
 * arrays: x unused; v (dim x N), w (dr x N), r, m, inertia (N),
 * f (dim x N), t (dr x N).  mu_c: per-contact friction or NULL.  R (dim x nc)
 * holds the starting forces on entry and the result on exit.
 * history (optional, 4 x max sweeps): n_pass, max_d_fail, r_avg, converged. */
int cdref_solve(const cdref_params* p, int64_t n, const double* v, const double* w,
                const double* r, const double* m, const double* inertia,
                const double* f, const double* t, const double* wall_velocity,
                int64_t nc, const int32_t* ci, const int32_t* cj,
                const double* normal, const double* gap, const double* mu_c,
                int P, const int64_t* dom_start, const int32_t* slot_contact,
                double* R, cdref_info* info, double* history);

/* Convergence tests of Sec. 2.1 after one sweep: Rprev = R^(j-1), R = R^j
 * (dim x nc), ravg_prev = R_avg^(j-1).  criterion 0 = local test (I),
 * 1 = global test (II).  Returns 1 when converged; also reports the count
 * passing the relative test, the largest |dR|^2 among the others, the new
 * R_avg and whether every force is finite. */
int cdref_criterion(int dim, int64_t nc, const double* Rprev, const double* R, double ravg_prev,
                    double alpha, int criterion, int64_t* n_pass, double* max_d_fail,
                    double* r_avg, int* finite);

/* Velocities from the contact forces (Eq. (1) and its rotational analogue). */
void cdref_velocities(int dim, int64_t n, double dt, const double* v, const double* w,
                      const double* m, const double* inertia, const double* r,
                      const double* f, const double* t, int64_t nc,
                      const int32_t* ci, const int32_t* cj, const double* normal,
                      const double* R, double* V, double* W);

/* Whole time steps with state carried between steps (Fig. 3 / Fig. 7). */
typedef struct cdref_sim cdref_sim;
cdref_sim* cdref_sim_create(const cdref_params* p, int64_t n, const double* x,
                            const double* v, const double* w, const double* r,
                            const double* m, const double* inertia, const double* f,
                            const double* t, const double* wall_normal,
                            const double* wall_offset, const double* wall_velocity,
                            const double* box_lo, const double* box_hi);
void cdref_sim_destroy(cdref_sim* s);
int cdref_sim_step(cdref_sim* s, cdref_info* info);
/* copies of the state: x, v (dim x N), w (dr x N), wall offsets (W) */
void cdref_sim_state(const cdref_sim* s, double* x, double* v, double* w, double* wall_offset);
/* the contacts of the last step: canonical list, forces, domains, order */
int64_t cdref_sim_contacts(const cdref_sim* s, int64_t cap, int32_t* ci, int32_t* cj,
                           double* normal, double* gap, double* R, int32_t* dom,
                           int32_t* color, int32_t* slot_contact);
/* mixed update from now on: contacts with pair number below p (p < 0: none) */
void cdref_sim_set_mixed(cdref_sim* s, double p, uint64_t seed);
/* random sequential order from now on (on = 0: colour-major); the step
 * index of the draws is the number of steps taken before */
int cdref_sim_set_random(cdref_sim* s, int on, uint64_t seed);
/* capacities (P doubles, domain order) used by every later tree rebuild;
 * NULL: back to leaf counts */
int cdref_sim_set_capacity(cdref_sim* s, const double* capacity);
/* Boundary conditions of the benchmark setups (Sec. 4.1, Sec. 4.4) from
 * now on: periodic_mask bit k makes axis k periodic with the box's length
 * (positions are kept in [lo, hi) on it, pairs taken at their nearest
 * image); wall_inv_mass (W, NULL: all 0) and wall_force (W, NULL: all 0)
 * give walls of finite mass 1/inv_mass pushed with the force along their
 * normal.  CDREF_EINVAL for a wall lying on a periodic axis. */
int cdref_sim_set_bc(cdref_sim* s, int periodic_mask, const double* wall_inv_mass,
                     const double* wall_force);
/* the walls' velocities after the steps so far (W x dim) */
void cdref_sim_wall_velocities(const cdref_sim* s, double* U);
/* The simulation box after the steps so far (dim entries each): a face
 * lying on an axis-aligned wall moves with that wall. */
void cdref_sim_box(const cdref_sim* s, double* lo, double* hi);
void cdref_sim_tree(const cdref_sim* s, int32_t* node_axis, double* node_cut,
                    int32_t* node_child, int32_t* node_leaf);

#ifdef __cplusplus
}
#endif
#endif
