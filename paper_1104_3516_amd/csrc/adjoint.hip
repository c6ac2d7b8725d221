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
  if (lb >= 0) {
    read_body<2>(sp, lb, B);
  } else {
    for (int q = 0; q < 3; ++q) B.V[q] = B.W[q] = 0.0;
    for (int q = 0; q < 2; ++q) B.V[q] = wu[(-1 - lb) * 2 + q];
    B.dm = B.di = B.r = 0.0;
  }
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
// those before it; returns the adjoint of its old force and dL/dmu.
__device__ inline void law_reverse(const SlotPre<2>& c, const double* tape, double rA,
                                   double dmA, double diA, double rB, double dmB, double diB,
                                   bool wall, const double* gR, double* ga, double* gb,
                                   double* gRold, double& gmu) {
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
  double gRn = gR[0] + gdRn, gRt = gR[1] + gdRt;   // total adjoint of the new force
  gRold[0] = -gdRn;
  gRold[1] = -gdRt;
  gmu = 0.0;
  double gs = 0.0, gut = 0.0;
  if (s < 0.0) {
    const double rn = -s * c.kn;
    const double T = -ut * c.kt;
    const double lim = c.mu * rn;
    if (fabs(T) <= lim) {
      gs = -c.kn * gRn;        // stick
      gut = -c.kt * gRt;
    } else {
      const double sg = T > 0.0 ? 1.0 : -1.0;   // slide: R_t = sign(T) mu R_n
      gmu = sg * rn * gRt;
      gs = -c.kn * (gRn + sg * c.mu * gRt);
    }
  }
  // u_n = v_n - dt w_n R_n,old ; u_t = v_t - dt w_t R_t,old
  gRold[0] = gRold[0] - c.dwn * gs;
  gRold[1] = gRold[1] - c.dwt * gut;
  const double gvn = gs, gvt = gut;
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
                                                              double* gmu_slot, int np_max) {
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
    gather_forces<2>(a, rin, e, rp, acc, tacc);
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
      fetch_slot<2>(a, rin, cs + k, c);
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
      fetch_slot<2>(a, rin, s, c);
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
      double gRold[2], gm;
      law_reverse(c, tape + 6 * (int64_t)k, rA, dmA, diA, rB, dmB, diB, wall, gR, ga, gb, gRold,
                  gm);
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
// (V = v + dt/m (f + sum of +-F), W = w + dt/I (t - sum r R_t))
__global__ __launch_bounds__(kT) void k_adjoint_contacts(int64_t nc, int64_t n,
                                                         const int* slot_contact, const int* ci,
                                                         const int* cj, const double* geo,
                                                         int64_t cap, const double* dtim,
                                                         const double* dtii, const double* r,
                                                         const double* own, const double* GV,
                                                         double* lam_out) {
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

}  // namespace

hipError_t cd_launch_mu_scatter(cd_ctx* c, const double* mu) {
  if (c->nc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mu_scatter, dim3(blocks_for(c->nc)), dim3(kT), 0, c->stream, mu,
                     c->contact_slot, c->nc, c->mu_slot);
  return hipGetLastError();
}

void cd_adjoint_release(cd_ctx* c) {
  AdjointWork* w = c->adj;
  if (!w) return;
  double** dptrs[] = {&w->lam[0], &w->lam[1], &w->own, &w->gE, &w->GV, &w->gv, &w->gmu, &w->seg};
  for (double** q : dptrs)
    if (*q) (void)hipFree(*q);
  int** iptrs[] = {&w->p2e_cnt, &w->p2e_ptr, &w->p2e};
  for (int** q : iptrs)
    if (*q) (void)hipFree(*q);
  if (w->state) (void)hipFree(w->state);
  delete w;
  c->adj = nullptr;
}

extern "C" {

int cd_adjoint(cd_ctx* c, const double* dL_dR, double* dL_dmu, double* dL_dv, double* dL_dw) {
  if (!c || !dL_dR) return CD_EINVAL;
  if (c->dim != 2) return cd_fail(c, CD_EINVAL, "the adjoint is implemented for 2D");
  if (!c->adj_valid || c->adj_K < 1)
    return cd_fail(c, CD_ENOTREADY,
                   "cd_adjoint needs a solve recorded with cd_set_adjoint and fixed_iters");
  if (c->sweep_global)
    return cd_fail(c, CD_ECAPACITY, "the adjoint needs every domain in LDS");
  const int64_t nc = c->nc, n = c->n, cap = c->cap, E = 2 * cap;
  const int C = c->adj_every, K = c->adj_K;
  hipStream_t st = c->stream;
  // LDS of the reverse sweep: particle records, tape, particle adjoints
  const int np_max = std::max(c->st_ds.max_particles, 1);
  const size_t lds = sizeof(double) * ((size_t)Layout<2>::PS * np_max + 6 * (size_t)c->st_ds.max_contacts +
                                       3 * (size_t)np_max);
  if (lds + 2048 > c->max_lds) return cd_fail(c, CD_ECAPACITY, "a domain is too large for the adjoint");
  if (!c->adj) c->adj = new AdjointWork();
  AdjointWork* w = c->adj;
  auto TRYH = [&](hipError_t e) { return e == hipSuccess ? CD_OK : cd_fail(c, CD_EHIP, hipGetErrorString(e)); };
#define ATRY(expr)                 \
  do {                             \
    int r_ = TRYH(expr);           \
    if (r_ != CD_OK) return r_;    \
  } while (0)
  if (w->cap < cap || w->n < n) {
    ATRY(alloc_n(&w->lam[0], 2 * cap));
    ATRY(alloc_n(&w->lam[1], 2 * cap));
    ATRY(alloc_n(&w->own, 2 * cap));
    ATRY(alloc_n(&w->gE, 3 * E));
    ATRY(alloc_n(&w->gmu, cap));
    ATRY(alloc_n(&w->GV, 3 * n));
    ATRY(alloc_n(&w->gv, 3 * n));
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
  if (!w->state) {
    ATRY(alloc_n(&w->state, 1));
    SolveState s0{};
    s0.done = 0;
    ATRY(hipMemcpy(w->state, &s0, sizeof(SolveState), hipMemcpyHostToDevice));
  }
  ATRY(hipMemsetAsync(w->gmu, 0, sizeof(double) * cap, st));
  ATRY(hipMemsetAsync(w->gv, 0, sizeof(double) * 3 * n, st));
  ATRY(hipMemsetAsync(w->gE, 0, sizeof(double) * 3 * E, st));
  if (nc > 0) {
    hipLaunchKernelGGL(k_lambda_init, dim3(blocks_for(nc)), dim3(kT), 0, st, dL_dR, c->contact_slot,
                       nc, w->lam[0]);
    ATRY(hipGetLastError());
  }
  // entries of each particle
  int dp_total = 0;
  ATRY(hipMemcpy(&dp_total, c->dp_start + c->P, sizeof(int), hipMemcpyDeviceToHost));
  ATRY(hipMemsetAsync(w->p2e_cnt, 0, sizeof(int) * (n + 1), st));
  hipLaunchKernelGGL(k_p2e_count, dim3(blocks_for(dp_total)), dim3(kT), 0, st, c->dp,
                     (int64_t)dp_total, w->p2e_cnt);
  ATRY(cd_scan_exclusive(c, w->p2e_cnt, w->p2e_ptr, n));
  ATRY(hipMemsetAsync(w->p2e_cnt, 0, sizeof(int) * (n + 1), st));
  hipLaunchKernelGGL(k_p2e_fill, dim3(blocks_for(dp_total)), dim3(kT), 0, st, c->dp,
                     (int64_t)dp_total, w->p2e_ptr, w->p2e_cnt, w->p2e);
  hipLaunchKernelGGL(k_p2e_sort, dim3(blocks_for(n)), dim3(kT), 0, st, n, w->p2e_ptr, w->p2e);
  ATRY(hipGetLastError());
  SweepArgs a = cd_sweep_args(c);
  const int block = c->sweep_block;
  const int S = (K + C - 1) / C;
  int cur = 0;   // lam[cur] holds the adjoint of R^k
  for (int sgi = S - 1; sgi >= 0; --sgi) {
    const int k0 = sgi * C, k1 = std::min(K, (sgi + 1) * C);
    const double* ck = c->ck + sgi * c->ck_stride;
    // forces R^(k0+1) .. R^(k1-1) of this segment, recomputed from R^k0
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
                         w->lam[cur], w->own, w->gE, w->gmu, np_max);
      hipLaunchKernelGGL(k_adjoint_particles, dim3(blocks_for(n)), dim3(kT), 0, st, n, w->p2e_ptr,
                         w->p2e, w->gE, w->GV, w->gv);
      if (nc > 0)
        hipLaunchKernelGGL(k_adjoint_contacts, dim3(blocks_for(nc)), dim3(kT), 0, st, nc, n,
                           c->slot_contact, c->ci, c->cj, c->geo, cap, c->dtim, c->dtii, c->r,
                           w->own, w->GV, w->lam[cur ^ 1]);
      ATRY(hipGetLastError());
      cur ^= 1;
    }
  }
  hipLaunchKernelGGL(k_adjoint_out, dim3(blocks_for(std::max(nc, n))), dim3(kT), 0, st, nc, n,
                     c->contact_slot, w->gmu, w->gv, dL_dmu, dL_dv, dL_dw);
  ATRY(hipGetLastError());
  ATRY(hipStreamSynchronize(st));
#undef ATRY
  return CD_OK;
}

}  // extern "C"
