// adjoint.hip - reverse mode of a recorded fixed-count solve (2D).
//
// The forward solve of a step is R^k = S(R^(k-1); v, w, mu) for k = 1..K,
// where S is one domain-wise sweep: every domain recomputes its particles'
// velocities from the base velocities and all forces R^(k-1) (exchange),
// then updates its native contacts colour by colour with the single-contact
// law (Sec. 2.1 and 3.1).  Given dL/dR^K, the reverse pass returns dL/dmu
// per contact and dL/dv, dL/dw of the velocities the step started from.
//
// Sweeps are reversed last to first.  The forces of the sweeps of one
// segment (between two checkpoints taken every adj_every sweeps during the
// forward solve) are recomputed from the segment's checkpoint with the
// forward sweep kernel itself, so they are bit-identical to the forward
// ones.  The reverse of sweep k runs one workgroup per domain:
//   1. it recomputes the domain's exchange and colour-by-colour update from
//      R^(k-1), keeping the body velocities each contact saw (the tape) in
//      LDS;
//   2. it walks the colours backwards: each contact's law is differentiated
//      in the branch it took (open: no dependence; stick: R_n = -(g_e/dt +
//      u_n)/(dt w_n), R_t = -u_t/(dt w_t); slide: R_t = sign(T) mu R_n), and
//      the adjoints of the domain's private velocities flow back;
//   3. the adjoints of the velocities at the domain's start are stored per
//      particle entry.
// Then, per particle, the entries' adjoints are summed in a fixed order
// (they are the adjoint of the base velocity for this sweep), and per
// contact the adjoint of R^(k-1) is its own-law part plus the exchange part
// from both bodies.  No atomics: the result does not depend on timing.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "sweep_core.h"

struct AdjointWork {
  double* lam[2] = {nullptr, nullptr};  // adjoint of R^k per slot: (R_n, R_t)
  double* own = nullptr;     // own-law part of the adjoint of R^(k-1), per slot
  double* gE = nullptr;      // per entry: adjoint of the domain-start velocity (V_x, V_y, W)
  double* GV = nullptr;      // per particle: sum over its entries (3 x N)
  double* gv = nullptr;      // per particle: accumulated dL/d(v, w) (3 x N)
  double* gmu = nullptr;     // per slot: accumulated dL/dmu
  double* seg = nullptr;     // recomputed records of one segment
  int* p2e_cnt = nullptr;    // entries of each particle (CSR)
  int* p2e_ptr = nullptr;
  int* p2e = nullptr;
  double* gn = nullptr;      // per slot: adjoint of the normal (2 x cap), this step
  double* ggdt = nullptr;    // per slot: adjoint of g_e/dt, this step
  double* gx = nullptr;      // per particle: adjoint of x^t (2 x N)
  double* gv_next = nullptr; // adjoints of v, w of the following step (3 x N)
  double* gx_next = nullptr; // adjoint of x of the following step (2 x N)
  double* gvt = nullptr;     // adjoint of v^(t+1) in full (2 x N)
  SolveState* state = nullptr;  // "open" state for the recomputing sweeps
  int64_t cap = 0, n = 0, seg_cap = 0;
};

namespace {

template <typename T>
hipError_t alloc_n(T** p, int64_t count) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  return hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
}

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void k_mu_scatter(const double* mu, const int* contact_slot,
                                                   int64_t nc, double* mu_slot) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c < nc) mu_slot[contact_slot[c]] = mu[c];
}

// adjoint of the final forces: canonical frame components -> slot order
__global__ __launch_bounds__(kT) void k_lambda_init(const double* dLdR, const int* contact_slot,
                                                    int64_t nc, double* lam) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= nc) return;
  const int64_t s = contact_slot[c];
  lam[2 * s] = dLdR[c];
  lam[2 * s + 1] = dLdR[nc + c];
}

// entries of each particle: count, then (after a scan) fill and sort by entry
__global__ __launch_bounds__(kT) void k_p2e_count(const int* dp, int64_t E, int* cnt) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e < E) atomicAdd(&cnt[dp[e]], 1);
}

__global__ __launch_bounds__(kT) void k_p2e_fill(const int* dp, int64_t E, const int* ptr,
                                                 int* cursor, int* p2e) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e < E) {
    const int p = dp[e];
    p2e[ptr[p] + atomicAdd(&cursor[p], 1)] = (int)e;
  }
}

__global__ __launch_bounds__(kT) void k_p2e_sort(int64_t n, const int* ptr, int* p2e) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  const int a = ptr[p], b = ptr[p + 1];
  for (int x = a + 1; x < b; ++x) {
    const int v = p2e[x];
    int y = x - 1;
    while (y >= a && p2e[y] > v) {
      p2e[y + 1] = p2e[y];
      --y;
    }
    p2e[y + 1] = v;
  }
}

// The forward part of one contact update with its body velocities before the
// update returned (the same arithmetic as update_contact).
__device__ inline void law_forward(double* sp, const double* wu, const SlotPre<2>& c, Body<2>& A,
                                   Body<2>& B) {
  const int la = c.ab.x, lb = c.ab.y;
  read_body<2>(sp, la, A);
  // body 2 chosen over scalars (a choice between two fillings of B's arrays
  // would be kept in scratch memory)
  const int lw = lb >= 0 ? lb : la;
  const double* pb = sp + (int64_t)Layout<2>::PS * lw;
  const double* pw = wu + 2 * (lb >= 0 ? 0 : -1 - lb);
  const bool part = lb >= 0;
  B.V[0] = part ? pb[0] : pw[0];
  B.V[1] = part ? pb[1] : pw[1];
  B.W[0] = part ? pb[Layout<2>::P_W] : 0.0;
  B.dm = part ? pb[Layout<2>::P_DM] : 0.0;
  B.di = part ? pb[Layout<2>::P_DI] : 0.0;
  B.r = part ? pb[Layout<2>::P_R] : 0.0;
  B.V[2] = B.W[1] = B.W[2] = 0.0;
  double nv[3] = {c.f[0], c.f[1], 0.0}, t1[3] = {-c.f[1], c.f[0], 0.0}, t2[3] = {0.0, 0.0, 0.0};
  double Rold[3] = {c.Ro[0], c.Ro[1], 0.0}, dwR[3] = {c.dwn * c.Ro[0], c.dwt * c.Ro[1], 0.0};
  double Rn[3] = {0.0, 0.0, 0.0};
  local_force<2>(nv, t1, t2, c.gdt, dwR, c.kn, c.kt, c.mu, A.r, B.r, A.V, A.W, B.V, B.W, Rn);
  const double dRn = Rn[0] - Rold[0], dR1 = Rn[1] - Rold[1];
  double dF[2];
  for (int q = 0; q < 2; ++q) dF[q] = dRn * nv[q] + dR1 * t1[q];
  double Va[3], Wa[3];
  for (int q = 0; q < 2; ++q) Va[q] = A.V[q] - A.dm * dF[q];
  Wa[0] = A.W[0] - A.di * (A.r * dR1);
  write_velocities<2>(sp, la, Va, Wa);
  if (lb >= 0) {
    double Vb[3], Wb[3];
    for (int q = 0; q < 2; ++q) Vb[q] = B.V[q] + B.dm * dF[q];
    Wb[0] = B.W[0] - B.di * (B.r * dR1);
    write_velocities<2>(sp, lb, Vb, Wb);
  }
}

// Reverse of one contact update.  tape: the body velocities it saw (V_a,
// W_a, V_b, W_b); gR: adjoint of its new force (R_n, R_t); ga, gb: adjoints
// of the bodies' velocities after the update (V_x, V_y, W), replaced by
// those before it; returns the adjoint of its old force, dL/dmu, and the
// adjoints of its normal (gn) and of g_e/dt (ggdt).
__device__ inline void law_reverse(const SlotPre<2>& c, const double* tape, double rA,
                                   double dmA, double diA, double rB, double dmB, double diB,
                                   bool wall, const double* gR, double* ga, double* gb,
                                   double* gRold, double& gmu, double* gn, double& ggdt) {
  const double n0 = c.f[0], n1 = c.f[1], t0 = -c.f[1], t1 = c.f[0];
  const double Va0 = tape[0], Va1 = tape[1], Wa = tape[2];
  const double Vb0 = tape[3], Vb1 = tape[4], Wb = tape[5];
  // forward quantities (the same operations as local_force)
  const double dV0 = Vb0 - Va0, dV1 = Vb1 - Va1;
  double vn = 0.0;
  vn = vn + dV0 * n0;
  vn = vn + dV1 * n1;
  const double dvt = dV0 * t0 + dV1 * t1;
  const double spin = rA * Wa + rB * Wb;
  const double vt = dvt - spin;
  const double un = vn - c.dwn * c.Ro[0];
  const double ut = vt - c.dwt * c.Ro[1];
  const double s = c.gdt + un;
  double Rn = 0.0, Rt = 0.0, sg = 0.0;
  bool stick = false;
  if (s < 0.0) {
    const double rn = -s * c.kn;
    const double T = -ut * c.kt;
    const double lim = c.mu * rn;
    Rn = rn;
    if (fabs(T) <= lim) {
      stick = true;
      Rt = T;
    } else {
      sg = T > 0.0 ? 1.0 : -1.0;
      Rt = T > 0.0 ? lim : -lim;
    }
  }
  const double dRn = Rn - c.Ro[0], dRt = Rt - c.Ro[1];
  // adjoint of the velocity updates (identity part kept in ga, gb)
  double gdF0 = -dmA * ga[0], gdF1 = -dmA * ga[1];
  double gdq = -diA * rA * ga[2];
  if (!wall) {
    gdF0 = gdF0 + dmB * gb[0];
    gdF1 = gdF1 + dmB * gb[1];
    gdq = gdq - diB * rB * gb[2];
  }
  const double gdRn = gdF0 * n0 + gdF1 * n1;
  const double gdRt = gdF0 * t0 + gdF1 * t1 + gdq;
  // dF = dR_n n + dR_t t with t = (-n_y, n_x)
  gn[0] = dRn * gdF0 + dRt * gdF1;
  gn[1] = -dRt * gdF0 + dRn * gdF1;
  const double gRn = gR[0] + gdRn, gRt = gR[1] + gdRt;   // total adjoint of the new force
  gRold[0] = -gdRn;
  gRold[1] = -gdRt;
  gmu = 0.0;
  double gs = 0.0, gut = 0.0;
  if (s < 0.0) {
    if (stick) {
      gs = -c.kn * gRn;        // R_n = -(g_e/dt + u_n)/(dt w_n), R_t = -u_t/(dt w_t)
      gut = -c.kt * gRt;
    } else {
      gmu = sg * Rn * gRt;     // slide: R_t = sign(T) mu R_n
      gs = -c.kn * (gRn + sg * c.mu * gRt);
    }
  }
  ggdt = gs;
  // u_n = v_n - dt w_n R_n,old ; u_t = v_t - dt w_t R_t,old
  gRold[0] = gRold[0] - c.dwn * gs;
  gRold[1] = gRold[1] - c.dwt * gut;
  const double gvn = gs, gvt = gut;
  // v_n = dV.n, v_t = dV.t - spin
  gn[0] = gn[0] + gvn * dV0 + gvt * dV1;
  gn[1] = gn[1] + gvn * dV1 - gvt * dV0;
  const double gspin = -gvt;
  const double gdV0 = gvn * n0 + gvt * t0, gdV1 = gvn * n1 + gvt * t1;
  ga[0] = ga[0] - gdV0;
  ga[1] = ga[1] - gdV1;
  ga[2] = ga[2] + rA * gspin;
  if (!wall) {
    gb[0] = gb[0] + gdV0;
    gb[1] = gb[1] + gdV1;
    gb[2] = gb[2] + rB * gspin;
  }
}

// Reverse of sweep k for one domain per workgroup (2D, LDS staging).
__global__ __launch_bounds__(kMaxBlock) void k_sweep_adjoint(SweepArgs a, const double* rin,
                                                              const double* lam_in,
                                                              double* own_out, double* gE,
                                                              double* gmu_slot, double* gn_slot,
                                                              double* ggdt_slot, int64_t cap,
                                                              int np_max) {
  using L = Layout<2>;
  constexpr int PS = L::PS;
  extern __shared__ double lds[];
  __shared__ int s_co[CD_MAX_COLORS + 1];
  __shared__ double s_wu[CD_MAX_WALLS * 3];
  const int d = domain_of(a, blockIdx.x, 0, a.grid / 8);
  if (d < 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int* dd = a.ddesc + 8 * (int64_t)d;
  const int cs = dd[0], nct = dd[1], ps = dd[2], np = dd[3], ncol = dd[4];
  double* sp = lds;                          // particle records [PS][np_max]
  double* tape = sp + (int64_t)PS * np_max;  // 6 doubles per slot
  double* gp = tape + 6 * (int64_t)nct;      // adjoints per particle: V_x, V_y, W
  const int* dcol = a.dcol + (int64_t)d * (CD_MAX_COLORS + 1);
  for (int q = tid; q <= ncol; q += nthr) s_co[q] = dcol[q];
  for (int q = tid; q < a.n_walls * 2; q += nthr) s_wu[q] = a.walls_u[q];
  // 1. exchange (as the forward sweep)
  const int64_t E = a.dpe;
  for (int l = tid; l < np; l += nthr) {
    const int64_t e = ps + l;
    double acc[2], tacc[1];
    for (int k = 0; k < 2; ++k) acc[k] = a.dpb[(3 + k) * E + e];
    tacc[0] = a.dpb[5 * E + e];
    const double dm = a.dpb[6 * E + e], di = a.dpb[7 * E + e], rp = a.dpb[8 * E + e];
    gather_forces<2>(a, rin, e, ((const int4*)a.drow)[e], rp, acc, tacc);
    double* pr = sp + (int64_t)PS * l;
    for (int k = 0; k < 2; ++k) pr[k] = a.dpb[k * E + e] + dm * acc[k];
    pr[L::P_W] = a.dpb[2 * E + e] + di * tacc[0];
    pr[L::P_DM] = dm;
    pr[L::P_DI] = di;
    pr[L::P_R] = rp;
    gp[3 * l] = gp[3 * l + 1] = gp[3 * l + 2] = 0.0;
  }
  __syncthreads();
  // 2a. forward colours with the tape
  for (int col = 0; col < ncol; ++col) {
    for (int k = s_co[col] + tid; k < s_co[col + 1]; k += nthr) {
      SlotPre<2> c;
      fetch_slot<2, true>(a, rin, cs + k, c);
      Body<2> A, B;
      law_forward(sp, s_wu, c, A, B);
      double* t = tape + 6 * (int64_t)k;
      t[0] = A.V[0];
      t[1] = A.V[1];
      t[2] = A.W[0];
      t[3] = B.V[0];
      t[4] = B.V[1];
      t[5] = B.W[0];
    }
    __syncthreads();
  }
  // 2b. colours backwards
  for (int col = ncol - 1; col >= 0; --col) {
    for (int k = s_co[col] + tid; k < s_co[col + 1]; k += nthr) {
      const int64_t s = cs + k;
      SlotPre<2> c;
      fetch_slot<2, true>(a, rin, s, c);
      const int la = c.ab.x, lb = c.ab.y;
      const bool wall = lb < 0;
      const double* pa = sp + (int64_t)PS * la;
      const double rA = pa[L::P_R], dmA = pa[L::P_DM], diA = pa[L::P_DI];
      double rB = 0.0, dmB = 0.0, diB = 0.0;
      if (!wall) {
        const double* pb = sp + (int64_t)PS * lb;
        rB = pb[L::P_R];
        dmB = pb[L::P_DM];
        diB = pb[L::P_DI];
      }
      double ga[3] = {gp[3 * la], gp[3 * la + 1], gp[3 * la + 2]};
      double gb[3] = {0.0, 0.0, 0.0};
      if (!wall)
        for (int q = 0; q < 3; ++q) gb[q] = gp[3 * lb + q];
      const double gR[2] = {lam_in[2 * s], lam_in[2 * s + 1]};
      double gRold[2], gm, gn[2], gg;
      law_reverse(c, tape + 6 * (int64_t)k, rA, dmA, diA, rB, dmB, diB, wall, gR, ga, gb, gRold,
                  gm, gn, gg);
      gn_slot[s] = gn_slot[s] + gn[0];
      gn_slot[cap + s] = gn_slot[cap + s] + gn[1];
      ggdt_slot[s] = ggdt_slot[s] + gg;
      for (int q = 0; q < 3; ++q) gp[3 * la + q] = ga[q];
      if (!wall)
        for (int q = 0; q < 3; ++q) gp[3 * lb + q] = gb[q];
      own_out[2 * s] = gRold[0];
      own_out[2 * s + 1] = gRold[1];
      gmu_slot[s] = gmu_slot[s] + gm;
    }
    __syncthreads();
  }
  // 3. adjoints of the domain-start velocities, per entry
  for (int l = tid; l < np; l += nthr) {
    const int64_t e = ps + l;
    for (int q = 0; q < 3; ++q) gE[3 * e + q] = gp[3 * l + q];
  }
}

// per particle: the entries' adjoints summed in entry order; accumulated
// into dL/d(v, w) (the base velocity enters every entry of every sweep)
__global__ __launch_bounds__(kT) void k_adjoint_particles(int64_t n, const int* ptr,
                                                          const int* p2e, const double* gE,
                                                          double* GV, double* gv) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  double g[3] = {0.0, 0.0, 0.0};
  for (int x = ptr[p]; x < ptr[p + 1]; ++x) {
    const int64_t e = p2e[x];
    for (int q = 0; q < 3; ++q) g[q] = g[q] + gE[3 * e + q];
  }
  for (int q = 0; q < 3; ++q) {
    GV[q * n + p] = g[q];
    gv[q * n + p] = gv[q * n + p] + g[q];
  }
}

// per slot: adjoint of R^(k-1) = own-law part + exchange part of both bodies
// (V = v + dt/m (f + sum of +-F), W = w + dt/I (t - sum r R_t)), and the
// exchange's share of the normal's adjoint (F = R_n n + R_t t)
__global__ __launch_bounds__(kT) void k_adjoint_contacts(int64_t nc, int64_t n,
                                                         const int* slot_contact, const int* ci,
                                                         const int* cj, const double* geo,
                                                         int64_t cap, const double* dtim,
                                                         const double* dtii, const double* r,
                                                         const double* own, const double* GV,
                                                         const double* rin, double* lam_out,
                                                         double* gn_slot) {
  const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (s >= nc) return;
  const int c = slot_contact[s];
  const int i = ci[c], j = cj[c];
  const double n0 = geo[G_N0 * cap + s], n1 = geo[(G_N0 + 1) * cap + s];
  const double t0 = -n1, t1 = n0;
  double gF0 = -dtim[i] * GV[i], gF1 = -dtim[i] * GV[n + i];
  double gRt = -dtii[i] * r[i] * GV[2 * n + i];
  if (j < n) {
    gF0 = gF0 + dtim[j] * GV[j];
    gF1 = gF1 + dtim[j] * GV[n + j];
    gRt = gRt - dtii[j] * r[j] * GV[2 * n + j];
  }
  lam_out[2 * s] = own[2 * s] + (gF0 * n0 + gF1 * n1);
  lam_out[2 * s + 1] = own[2 * s + 1] + ((gF0 * t0 + gF1 * t1) + gRt);
  const double Rn = rin[4 * s], Rt = rin[4 * s + 1];
  gn_slot[s] = gn_slot[s] + (Rn * gF0 + Rt * gF1);
  gn_slot[cap + s] = gn_slot[cap + s] + (-Rt * gF0 + Rn * gF1);
}

// ---- between time steps (frozen contact list) -----------------------------

// the kept list at new positions: slot normals and g_e/dt, the previous
// step's canonical forces as the starting records (the world force with the
// new normal, as the order stage writes them)
__global__ __launch_bounds__(kT) void k_frozen_refresh(int64_t nc, const int* slot_contact,
                                                       const double* nrm, const double* gap,
                                                       const double* R, double dt, int clamp,
                                                       double* geo, int64_t cap, double* rec0) {
  const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (s >= nc) return;
  const int c = slot_contact[s];
  const double n0 = nrm[c], n1 = nrm[nc + c];
  double ge = gap[c];
  if (clamp && ge < 0.0) ge = 0.0;
  geo[G_N0 * cap + s] = n0;
  geo[(G_N0 + 1) * cap + s] = n1;
  geo[G_GDT * cap + s] = ge / dt;
  const double rn = R[c], r1 = R[nc + c];
  const double t0 = -n1, t1 = n0;
  double* rc = rec0 + 4 * s;
  rc[0] = rn;
  rc[1] = r1;
  rc[2] = rn * n0 + r1 * t0;
  rc[3] = rn * n1 + r1 * t1;
}

// base velocities of the domain particle entries (rows v_x, v_y, w)
__global__ __launch_bounds__(kT) void k_dpb_base(const int* dp, const int* dp_start, int P,
                                                 int64_t E, const double* v, const double* w,
                                                 int64_t n, double* dpb) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= E || e >= dp_start[P]) return;
  const int p = dp[e];
  dpb[e] = v[p];
  dpb[E + e] = v[n + p];
  dpb[2 * E + e] = w[p];
}

// slot geometry of a recorded step back into the slot constants
__global__ __launch_bounds__(kT) void k_restore_geo(int64_t nc, const double* gn, const double* gdt,
                                                    double* geo, int64_t cap) {
  const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (s >= nc) return;
  geo[G_N0 * cap + s] = gn[s];
  geo[(G_N0 + 1) * cap + s] = gn[cap + s];
  geo[G_GDT * cap + s] = gdt[s];
}

// adjoint of v^(t+1) in full: from the next step's base velocity and, through
// x^(t+1) = x^t + dt v^(t+1), from the next step's positions
__global__ __launch_bounds__(kT) void k_euler_prep(int64_t n, double dt, const double* gv_next,
                                                   const double* gx_next, double* gvt) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  gvt[p] = gv_next[p] + dt * gx_next[p];
  gvt[n + p] = gv_next[n + p] + dt * gx_next[n + p];
}

// reverse of the velocity update v^(t+1) = v^t + dt/m (f + sum +-F(R^K)),
// w^(t+1) = w^t + dt/I (t - sum r R_t): adds to the adjoint of the final
// forces and of the normals of step t
__global__ __launch_bounds__(kT) void k_euler_reverse(int64_t nc, int64_t n,
                                                      const int* slot_contact, const int* ci,
                                                      const int* cj, const double* geo,
                                                      int64_t cap, const double* dtim,
                                                      const double* dtii, const double* r,
                                                      const double* gvt, const double* gw_next,
                                                      const double* fin, double* lam,
                                                      double* gn_slot) {
  const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (s >= nc) return;
  const int c = slot_contact[s];
  const int i = ci[c], j = cj[c];
  const double n0 = geo[G_N0 * cap + s], n1 = geo[(G_N0 + 1) * cap + s];
  double gF0 = -dtim[i] * gvt[i], gF1 = -dtim[i] * gvt[n + i];
  double gRt = -dtii[i] * r[i] * gw_next[i];
  if (j < n) {
    gF0 = gF0 + dtim[j] * gvt[j];
    gF1 = gF1 + dtim[j] * gvt[n + j];
    gRt = gRt - dtii[j] * r[j] * gw_next[j];
  }
  lam[2 * s] = lam[2 * s] + (gF0 * n0 + gF1 * n1);
  lam[2 * s + 1] = lam[2 * s + 1] + ((gF0 * -n1 + gF1 * n0) + gRt);
  const double Rn = fin[4 * s], Rt = fin[4 * s + 1];
  gn_slot[s] = gn_slot[s] + (Rn * gF0 + Rt * gF1);
  gn_slot[cap + s] = gn_slot[cap + s] + (-Rt * gF0 + Rn * gF1);
}

// reverse of the geometry of step t per particle, over its contacts in
// ascending id: n = d/|d|, g = |d| - r_i - r_j with d = x_j - x_i, or for a
// wall n = -nu, g = nu.x_i - o - r_i; g_e = max(g, 0) (clamped) or g
__global__ __launch_bounds__(kT) void k_geom_reverse(int64_t n, const int* inc_ptr, const int* inc,
                                                     const int* slot_contact, const int* ci,
                                                     const int* cj, const double* x,
                                                     const double* wall, const double* gap,
                                                     int64_t cap, double dt, int clamp,
                                                     const double* gn_slot,
                                                     const double* ggdt_slot, double* gx) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= n) return;
  double g0 = 0.0, g1 = 0.0;
  for (int e = inc_ptr[p]; e < inc_ptr[p + 1]; ++e) {
    const int ent = inc[e];
    const int64_t s = ent >> 1;
    const int c = slot_contact[s];
    const int i = ci[c], j = cj[c];
    const double gg = (clamp && !(gap[c] > 0.0)) ? 0.0 : ggdt_slot[s] / dt;
    if (j < n) {
      const double d0 = x[j] - x[i], d1 = x[n + j] - x[n + i];
      const double dist = sqrt(d0 * d0 + d1 * d1);
      const double m0 = d0 / dist, m1 = d1 / dist;
      const double ln0 = gn_slot[s], ln1 = gn_slot[cap + s];
      const double proj = m0 * ln0 + m1 * ln1;
      const double gd0 = (ln0 - m0 * proj) / dist + m0 * gg;
      const double gd1 = (ln1 - m1 * proj) / dist + m1 * gg;
      if (ent & 1) {
        g0 = g0 + gd0;
        g1 = g1 + gd1;
      } else {
        g0 = g0 - gd0;
        g1 = g1 - gd1;
      }
    } else {
      const double* nu = wall + 2 * (j - n);
      g0 = g0 + nu[0] * gg;
      g1 = g1 + nu[1] * gg;
    }
  }
  gx[p] = gx[p] + g0;
  gx[n + p] = gx[n + p] + g1;
}

__global__ __launch_bounds__(kT) void k_adjoint_out(int64_t nc, int64_t n, const int* contact_slot,
                                                    const double* gmu_slot, const double* gv,
                                                    double* dLdmu, double* dLdv, double* dLdw) {
  const int64_t x = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (dLdmu && x < nc) dLdmu[x] = gmu_slot[contact_slot[x]];
  if (x < n) {
    if (dLdv) {
      dLdv[x] = gv[x];
      dLdv[n + x] = gv[n + x];
    }
    if (dLdw) dLdw[x] = gv[2 * n + x];
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, (n + kT - 1) / kT); }

// zeroes `words` 4-byte words (every buffer cleared here is a whole number of them)
__global__ __launch_bounds__(kT) void k_zero_words(unsigned* p, int64_t words) {
  const int64_t x = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (x < words) p[x] = 0u;
}

}  // namespace

hipError_t cd_launch_mu_scatter(cd_ctx* c, const double* mu) {
  if (c->nc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mu_scatter, dim3(blocks_for(c->nc)), dim3(kT), 0, c->stream, mu,
                     c->contact_slot, c->nc, c->mu_slot);
  return hipGetLastError();
}

hipError_t cd_launch_frozen_refresh(cd_ctx* c) {
  if (c->nc > 0)
    hipLaunchKernelGGL(k_frozen_refresh, dim3(blocks_for(c->nc)), dim3(kT), 0, c->stream, c->nc,
                       c->slot_contact, c->nrm, c->gap, c->R, c->p.dt, c->p.overlap_mode == 0,
                       c->geo, c->cap, c->rec[0]);
  const int64_t E = 2 * c->cap;
  if (c->dim == 2) {
    hipLaunchKernelGGL(k_dpb_base, dim3(blocks_for(E)), dim3(kT), 0, c->stream, c->dp,
                       c->dp_start, c->P, E, c->v, c->w, c->n, c->dpb);
  } else {
    return hipErrorInvalidValue;   // kept lists are 2D (the adjoint's case)
  }
  return hipGetLastError();
}

void cd_window_clear(cd_ctx* c) {
  for (auto& r : c->win) {
    double* ptrs[] = {r.x, r.v, r.w, r.geo_n, r.geo_gdt, r.gap, r.ck, r.fin};
    for (double* q : ptrs)
      if (q) (void)hipFree(q);
  }
  c->win.clear();
}

int cd_window_begin(cd_ctx* c) {
  c->win.emplace_back();
  cd_ctx::StepRec& r = c->win.back();
  const int64_t n = c->n;
  if (alloc_n(&r.x, c->dim * n) != hipSuccess || alloc_n(&r.v, c->dim * n) != hipSuccess ||
      alloc_n(&r.w, c->dr * n) != hipSuccess)
    return cd_fail(c, CD_ENOMEM, "adjoint window: out of device memory");
  const size_t b = sizeof(double) * (size_t)n;
  if (hipMemcpyAsync(r.x, c->x, b * c->dim, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(r.v, c->v, b * c->dim, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(r.w, c->w, b * c->dr, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return cd_fail(c, CD_EHIP, "adjoint window: copy failed");
  return CD_OK;
}

int cd_window_geometry(cd_ctx* c) {
  if (c->win.empty()) return CD_OK;
  cd_ctx::StepRec& r = c->win.back();
  const int64_t cap = c->cap, nc = c->nc;
  if (alloc_n(&r.geo_n, 2 * cap) != hipSuccess || alloc_n(&r.geo_gdt, cap) != hipSuccess ||
      alloc_n(&r.gap, nc) != hipSuccess)
    return cd_fail(c, CD_ENOMEM, "adjoint window: out of device memory");
  const size_t b = sizeof(double);
  if (hipMemcpyAsync(r.geo_n, c->geo + G_N0 * cap, b * 2 * cap, hipMemcpyDeviceToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(r.geo_gdt, c->geo + G_GDT * cap, b * cap, hipMemcpyDeviceToDevice,
                     c->stream) != hipSuccess ||
      (nc > 0 && hipMemcpyAsync(r.gap, c->gap, b * nc, hipMemcpyDeviceToDevice, c->stream) !=
                     hipSuccess))
    return cd_fail(c, CD_EHIP, "adjoint window: copy failed");
  return CD_OK;
}

void cd_adjoint_release(cd_ctx* c) {
  AdjointWork* w = c->adj;
  if (!w) return;
  double** dptrs[] = {&w->lam[0], &w->lam[1], &w->own, &w->gE, &w->GV, &w->gv, &w->gmu, &w->seg,
                      &w->gn, &w->ggdt, &w->gx, &w->gv_next, &w->gx_next, &w->gvt};
  for (double** q : dptrs)
    if (*q) (void)hipFree(*q);
  int** iptrs[] = {&w->p2e_cnt, &w->p2e_ptr, &w->p2e};
  for (int** q : iptrs)
    if (*q) (void)hipFree(*q);
  if (w->state) (void)hipFree(w->state);
  delete w;
  c->adj = nullptr;
}

// ---- allocation-free variant (cd_adjoint_static) --------------------------
// The reverse pass's workspace carved from one file-scope device array per
// GPU instead of hipMalloc'ed buffers.  Each device holds its own copy from
// the module's load until the process ends; its address comes from
// hipGetSymbolAddress with that device current, once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (nullptr on failure)
int scratch_address(cd_ctx* c, unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return cd_fail(c, CD_EHIP, "no current device for the static workspace");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cd_fail(c, CD_EHIP, "hipGetSymbolAddress of the static workspace failed");
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return CD_OK;
}

// Bytes of the reverse pass's workspace for this context and its layout in a
// block at `base` (nullptr: size only), 256-byte aligned pieces.
size_t carve_work(AdjointWork* w, unsigned char* base, int64_t cap, int64_t n, int C) {
  const int64_t E = 2 * cap;
  size_t off = 0;
  auto take = [&](auto** p, int64_t count, size_t elem) {
    const size_t bytes = ((size_t)std::max<int64_t>(count, 1) * elem + 255) / 256 * 256;
    if (base) *p = (std::remove_reference_t<decltype(**p)>*)(base + off);
    off += bytes;
  };
  take(&w->lam[0], 2 * cap, sizeof(double));
  take(&w->lam[1], 2 * cap, sizeof(double));
  take(&w->own, 2 * cap, sizeof(double));
  take(&w->gE, 3 * E, sizeof(double));
  take(&w->gmu, cap, sizeof(double));
  take(&w->gn, 2 * cap, sizeof(double));
  take(&w->ggdt, cap, sizeof(double));
  take(&w->GV, 3 * n, sizeof(double));
  take(&w->gv, 3 * n, sizeof(double));
  take(&w->gx, 2 * n, sizeof(double));
  take(&w->gv_next, 3 * n, sizeof(double));
  take(&w->gx_next, 2 * n, sizeof(double));
  take(&w->gvt, 2 * n, sizeof(double));
  take(&w->p2e_cnt, n + 1, sizeof(int));
  take(&w->p2e_ptr, n + 1, sizeof(int));
  take(&w->p2e, E, sizeof(int));
  take(&w->seg, (int64_t)C * 4 * cap, sizeof(double));
  take(&w->state, 1, sizeof(SolveState));
  if (base) {
    w->cap = cap;
    w->n = n;
    w->seg_cap = (int64_t)C * 4 * cap;
  }
  return off;
}

}  // namespace

// Reverse of every step of the recorded window, last to first.  For step t:
// the Euler update's reverse (from the adjoints of x, v, w at step t+1), the
// solve's reverse (seeded with the adjoint of its final forces), the
// geometry's reverse; the adjoint of the step's starting forces (its warm
// start) seeds the previous step's final forces.  `fixed`: the workspace w
// is in place already (the static variant) and nothing is allocated here.
static int adjoint_run(cd_ctx* c, AdjointWork* w, bool fixed, const double* dL_dR,
                       double* dL_dmu, double* dL_dv, double* dL_dw) {
  const int64_t nc = c->nc, n = c->n, cap = c->cap, E = 2 * cap;
  const int C = c->adj_every;
  const int T = (int)c->win.size();
  const double dt = c->p.dt;
  const int clamp = c->p.overlap_mode == 0;
  hipStream_t st = c->stream;
  const int np_max = std::max(c->st_ds.max_particles, 1);
  const size_t lds = sizeof(double) * ((size_t)Layout<2>::PS * np_max +
                                       6 * (size_t)c->st_ds.max_contacts + 3 * (size_t)np_max);
  auto TRYH = [&](hipError_t e) {
    return e == hipSuccess ? CD_OK : cd_fail(c, CD_EHIP, hipGetErrorString(e));
  };
#define ATRY(expr)              \
  do {                          \
    int r_ = TRYH(expr);        \
    if (r_ != CD_OK) return r_; \
  } while (0)
  // zeroed with a fill kernel (no memset nodes if a caller captures the stream)
  auto zero = [&](void* p, size_t bytes) {
    const int64_t words = (int64_t)(bytes / sizeof(unsigned));
    if (words > 0)
      hipLaunchKernelGGL(k_zero_words, dim3(blocks_for(words)), dim3(kT), 0, st, (unsigned*)p,
                         words);
    return hipGetLastError();
  };
  if (!fixed) {
    if (w->cap < cap || w->n < n) {
      ATRY(alloc_n(&w->lam[0], 2 * cap));
      ATRY(alloc_n(&w->lam[1], 2 * cap));
      ATRY(alloc_n(&w->own, 2 * cap));
      ATRY(alloc_n(&w->gE, 3 * E));
      ATRY(alloc_n(&w->gmu, cap));
      ATRY(alloc_n(&w->gn, 2 * cap));
      ATRY(alloc_n(&w->ggdt, cap));
      ATRY(alloc_n(&w->GV, 3 * n));
      ATRY(alloc_n(&w->gv, 3 * n));
      ATRY(alloc_n(&w->gx, 2 * n));
      ATRY(alloc_n(&w->gv_next, 3 * n));
      ATRY(alloc_n(&w->gx_next, 2 * n));
      ATRY(alloc_n(&w->gvt, 2 * n));
      ATRY(alloc_n(&w->p2e_cnt, n + 1));
      ATRY(alloc_n(&w->p2e_ptr, n + 1));
      ATRY(alloc_n(&w->p2e, E));
      w->cap = cap;
      w->n = n;
    }
    if (w->seg_cap < (int64_t)C * 4 * cap) {
      ATRY(alloc_n(&w->seg, (int64_t)C * 4 * cap));
      w->seg_cap = (int64_t)C * 4 * cap;
    }
    if (!w->state) ATRY(alloc_n(&w->state, 1));
  }
  // the recomputing sweeps run "open" (done = 0): a zeroed state
  ATRY(zero(w->state, sizeof(SolveState)));
  ATRY(zero(w->gmu, sizeof(double) * cap));
  ATRY(zero(w->gE, sizeof(double) * 3 * E));
  ATRY(zero(w->gv_next, sizeof(double) * 3 * n));
  ATRY(zero(w->gx_next, sizeof(double) * 2 * n));
  ATRY(zero(w->lam[0], sizeof(double) * 2 * cap));
  if (nc > 0) {
    hipLaunchKernelGGL(k_lambda_init, dim3(blocks_for(nc)), dim3(kT), 0, st, dL_dR,
                       c->contact_slot, nc, w->lam[0]);
    ATRY(hipGetLastError());
  }
  // entries of each particle (the same for every step of the window); the
  // count comes back through the pinned scratch
  ATRY(hipMemcpyAsync(c->h_scratch, c->dp_start + c->P, sizeof(int), hipMemcpyDeviceToHost, st));
  ATRY(hipStreamSynchronize(st));
  const int dp_total = ((const int*)c->h_scratch)[0];
  ATRY(zero(w->p2e_cnt, sizeof(int) * (n + 1)));
  hipLaunchKernelGGL(k_p2e_count, dim3(blocks_for(dp_total)), dim3(kT), 0, st, c->dp,
                     (int64_t)dp_total, w->p2e_cnt);
  ATRY(cd_scan_exclusive(c, w->p2e_cnt, w->p2e_ptr, n));
  ATRY(zero(w->p2e_cnt, sizeof(int) * (n + 1)));
  hipLaunchKernelGGL(k_p2e_fill, dim3(blocks_for(dp_total)), dim3(kT), 0, st, c->dp,
                     (int64_t)dp_total, w->p2e_ptr, w->p2e_cnt, w->p2e);
  hipLaunchKernelGGL(k_p2e_sort, dim3(blocks_for(n)), dim3(kT), 0, st, n, w->p2e_ptr, w->p2e);
  ATRY(hipGetLastError());
  const int block = c->sweep_block;
  int cur = 0;   // lam[cur] holds the adjoint of the forces being reversed
  for (int t = T - 1; t >= 0; --t) {
    const cd_ctx::StepRec& r = c->win[t];
    const int K = r.K;
    // the step's geometry and base velocities back in place
    if (nc > 0)
      hipLaunchKernelGGL(k_restore_geo, dim3(blocks_for(nc)), dim3(kT), 0, st, nc, r.geo_n,
                         r.geo_gdt, c->geo, cap);
    hipLaunchKernelGGL(k_dpb_base, dim3(blocks_for(E)), dim3(kT), 0, st, c->dp, c->dp_start, c->P,
                       E, r.v, r.w, n, c->dpb);
    ATRY(hipGetLastError());
    ATRY(zero(w->gv, sizeof(double) * 3 * n));
    ATRY(zero(w->gn, sizeof(double) * 2 * cap));
    ATRY(zero(w->ggdt, sizeof(double) * cap));
    // the Euler update of step t (x, v, w of step t+1 depend on its forces)
    if (t < T - 1) {
      hipLaunchKernelGGL(k_euler_prep, dim3(blocks_for(n)), dim3(kT), 0, st, n, dt, w->gv_next,
                         w->gx_next, w->gvt);
      if (nc > 0)
        hipLaunchKernelGGL(k_euler_reverse, dim3(blocks_for(nc)), dim3(kT), 0, st, nc, n,
                           c->slot_contact, c->ci, c->cj, c->geo, cap, c->dtim, c->dtii, c->r,
                           w->gvt, w->gv_next + 2 * n, r.fin, w->lam[cur], w->gn);
      ATRY(hipGetLastError());
      // v^t and w^t pass into v^(t+1), w^(t+1) unchanged; x^t into x^(t+1)
      ATRY(hipMemcpyAsync(w->gv, w->gvt, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st));
      ATRY(hipMemcpyAsync(w->gv + 2 * n, w->gv_next + 2 * n, sizeof(double) * n,
                          hipMemcpyDeviceToDevice, st));
      ATRY(hipMemcpyAsync(w->gx, w->gx_next, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice,
                          st));
    } else {
      ATRY(zero(w->gx, sizeof(double) * 2 * n));
    }
    // the solve of step t, sweep by sweep from the last
    SweepArgs a = cd_sweep_args(c);
    const int S = (K + C - 1) / C;
    for (int sgi = S - 1; sgi >= 0; --sgi) {
      const int k0 = sgi * C, k1 = std::min(K, (sgi + 1) * C);
      const double* ck = r.ck + sgi * c->ck_stride;
      auto R_of = [&](int k) -> const double* {
        return k == k0 ? ck : w->seg + (int64_t)(k - k0 - 1) * 4 * cap;
      };
      for (int k = k0 + 1; k < k1; ++k) {
        SweepArgs f = a;
        f.rec[(k - 1) & 1] = const_cast<double*>(R_of(k - 1));
        f.rec[k & 1] = w->seg + (int64_t)(k - k0 - 1) * 4 * cap;
        f.state = w->state;
        ATRY(cd_launch_sweep_grid(c, f, k, f.grid));
      }
      for (int k = k1; k > k0; --k) {
        hipLaunchKernelGGL(k_sweep_adjoint, dim3(a.grid), dim3(block), lds, st, a, R_of(k - 1),
                           w->lam[cur], w->own, w->gE, w->gmu, w->gn, w->ggdt, cap, np_max);
        hipLaunchKernelGGL(k_adjoint_particles, dim3(blocks_for(n)), dim3(kT), 0, st, n,
                           w->p2e_ptr, w->p2e, w->gE, w->GV, w->gv);
        if (nc > 0)
          hipLaunchKernelGGL(k_adjoint_contacts, dim3(blocks_for(nc)), dim3(kT), 0, st, nc, n,
                             c->slot_contact, c->ci, c->cj, c->geo, cap, c->dtim, c->dtii, c->r,
                             w->own, w->GV, R_of(k - 1), w->lam[cur ^ 1], w->gn);
        ATRY(hipGetLastError());
        cur ^= 1;
      }
    }
    // the geometry of step t
    hipLaunchKernelGGL(k_geom_reverse, dim3(blocks_for(n)), dim3(kT), 0, st, n, c->inc_ptr,
                       c->inc, c->slot_contact, c->ci, c->cj, r.x, c->d_wall, r.gap, cap, dt,
                       clamp, w->gn, w->ggdt, w->gx);
    ATRY(hipGetLastError());
    // adjoints of x^t, v^t, w^t for the step before
    ATRY(hipMemcpyAsync(w->gv_next, w->gv, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
    ATRY(hipMemcpyAsync(w->gx_next, w->gx, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, st));
    // lam[cur] now holds the adjoint of step t's starting forces = step t-1's final forces
  }
  hipLaunchKernelGGL(k_adjoint_out, dim3(blocks_for(std::max(nc, n))), dim3(kT), 0, st, nc, n,
                     c->contact_slot, w->gmu, w->gv, dL_dmu, dL_dv, dL_dw);
  ATRY(hipGetLastError());
  ATRY(hipStreamSynchronize(st));
#undef ATRY
  return CD_OK;
}

// The checks both entry points make before any work.
static int adjoint_check(cd_ctx* c, const double* dL_dR) {
  if (!c || !dL_dR) return CD_EINVAL;
  if (c->dim != 2) return cd_fail(c, CD_EINVAL, "the adjoint is implemented for 2D");
  if (!c->adj_valid || c->win.empty() || c->win.back().K < 1)
    return cd_fail(c, CD_ENOTREADY,
                   "cd_adjoint needs a solve recorded with cd_set_adjoint and fixed_iters");
  if (c->sweep_global)
    return cd_fail(c, CD_ECAPACITY, "the adjoint needs every domain in LDS");
  const int np_max = std::max(c->st_ds.max_particles, 1);
  const size_t lds = sizeof(double) * ((size_t)Layout<2>::PS * np_max +
                                       6 * (size_t)c->st_ds.max_contacts + 3 * (size_t)np_max);
  if (lds + 2048 > c->max_lds)
    return cd_fail(c, CD_ECAPACITY, "a domain is too large for the adjoint");
  return CD_OK;
}

extern "C" {

int cd_adjoint(cd_ctx* c, const double* dL_dR, double* dL_dmu, double* dL_dv, double* dL_dw) {
  const int st = adjoint_check(c, dL_dR);
  if (st != CD_OK) return st;
  if (!c->adj) c->adj = new AdjointWork();
  return adjoint_run(c, c->adj, false, dL_dR, dL_dmu, dL_dv, dL_dw);
}

int cd_adjoint_static(cd_ctx* c, const double* dL_dR, double* dL_dmu, double* dL_dv,
                      double* dL_dw) {
  int st = adjoint_check(c, dL_dR);
  if (st != CD_OK) return st;
  AdjointWork w;
  const size_t need = carve_work(&w, nullptr, c->cap, c->n, c->adj_every);
  if (need > kScratchBytes)
    return cd_fail(c, CD_ECAPACITY,
                   "cd_adjoint_static: the workspace exceeds the 64 MiB static array "
                   "(fewer contacts or particles, or a shorter checkpoint interval)");
  // the prefix scan's status words belong to the context; the forward steps
  // sized them for at least n + 1 entries, which is checked here
  if (c->scan_tmp_cap < (c->n + 2048 - 1) / 2048 + 1)
    return cd_fail(c, CD_ECAPACITY, "cd_adjoint_static: scan workspace not sized by a step");
  unsigned char* base = nullptr;
  st = scratch_address(c, &base);
  if (st != CD_OK) return st;
  carve_work(&w, base, c->cap, c->n, c->adj_every);
  return adjoint_run(c, &w, true, dL_dR, dL_dmu, dL_dv, dL_dw);
}

}  // extern "C"
