// sweep_core.h - device helpers of the domain sweep shared by the forward
// sweep kernels (sweep.hip) and their adjoint (adjoint.hip): the staging
// layout, the single-contact law, the exchange gathers and the update of one
// contact.  Everything is inline and internal to each including file.
#pragma once
#include "cd_internal.h"

namespace {

template <int DIM>
struct Layout {
  static constexpr int DR = DIM == 2 ? 1 : 3;
  static constexpr int REC = cd_rec(DIM);
  static constexpr int NG = DIM == 2 ? 2 : 9;      // frame doubles per slot
  static constexpr int NGS = DIM == 2 ? 2 : 3;     // of which staged in LDS (the normal)
  // staged particle record (doubles): V [0, DIM), W [DIM, DIM+DR), dt/m, dt/I,
  // r, padded to an even count so that pairs load as 16-byte words
  static constexpr int PS = cd_stage_particle(DIM);
  static constexpr int P_W = DIM, P_DM = DIM + DR, P_DI = DIM + DR + 1, P_R = DIM + DR + 2;
  static_assert(P_R < PS && PS % 2 == 0, "particle staging layout");
};

// The single-contact law (Eqs. 3-9, Fig. 2) for the contact's frame n, t1,
// t2 and the body velocities; dwR = (dt w_n R_n, dt w_t R_t1, dt w_t R_t2) of
// the contact's current force removes that force's own share of the relative
// velocity.  Writes the new frame force.
template <int DIM>
__device__ inline void local_force(const double* n, const double* t1, const double* t2, double gdt,
                                   const double* dwR, double kn, double kt, double mu, double ra,
                                   double rb, const double* Va, const double* Wa, const double* Vb,
                                   const double* Wb, double* Rnew) {
  double dV[3];
  for (int q = 0; q < DIM; ++q) dV[q] = Vb[q] - Va[q];
  double vn = 0.0;
  for (int q = 0; q < DIM; ++q) vn = vn + dV[q] * n[q];
  double vt1, vt2 = 0.0;
  if (DIM == 2) {
    double dvt = dV[0] * t1[0] + dV[1] * t1[1];
    double spin = ra * Wa[0] + rb * Wb[0];
    vt1 = dvt - spin;
  } else {
    double spin[3];
    for (int q = 0; q < 3; ++q) spin[q] = ra * Wa[q] + rb * Wb[q];
    double dvt1 = 0.0, dvt2 = 0.0, s2 = 0.0, s1 = 0.0;
    for (int q = 0; q < 3; ++q) {
      dvt1 = dvt1 + dV[q] * t1[q];
      dvt2 = dvt2 + dV[q] * t2[q];
      s2 = s2 + spin[q] * t2[q];
      s1 = s1 + spin[q] * t1[q];
    }
    vt1 = dvt1 - s2;
    vt2 = dvt2 + s1;
  }
  // relative velocity the pair would have without this contact's force
  double un = vn - dwR[0];
  double ut1 = vt1 - dwR[1];
  double ut2 = DIM == 3 ? vt2 - dwR[DIM - 1] : 0.0;
  double s = gdt + un;      // predicted gap / dt (Eq. 3)
  Rnew[0] = 0.0;
  Rnew[1] = 0.0;
  if (DIM == 3) Rnew[2] = 0.0;
  if (s >= 0.0) return;     // stays open
  double rn = -s * kn;      // sticking force, normal part (Eqs. 4-5)
  double T1 = -ut1 * kt;
  double T2 = DIM == 3 ? -ut2 * kt : 0.0;
  double lim = mu * rn;     // Coulomb bound (Eq. 7)
  Rnew[0] = rn;
  if (DIM == 2) {
    if (fabs(T1) <= lim) Rnew[1] = T1;
    else Rnew[1] = T1 > 0.0 ? lim : -lim;   // sliding (Eqs. 8-9)
  } else {
    double tn = sqrt(T1 * T1 + T2 * T2);
    if (tn <= lim) {
      Rnew[1] = T1;
      Rnew[2] = T2;
    } else {
      double fac = lim / tn;
      Rnew[1] = T1 * fac;
      Rnew[2] = T2 * fac;
    }
  }
}

constexpr int kMaxBlock = 256;
// s_waitcnt immediate (gfx9 encoding) waiting for vmcnt = 0 only
constexpr int kWaitVm0 = 0x0F70;

// Workgroup barrier ordering LDS only: unlike __syncthreads it does not wait
// for the wave's outstanding global loads and stores.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders the calling wavefront's LDS writes before its later LDS reads (for
// the compiler only: the hardware completes a wavefront's LDS operations in
// issue order, so no wait is needed).
__device__ inline void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// four doubles stored with one streaming (non-temporal) 32-byte store
typedef double nt4 __attribute__((ext_vector_type(4)));

// The domain of block b in pass k.  Block b runs on XCD x = b % 8
// (round-robin dispatch); XCD x owns the contiguous domain range
// [x per, (x+1) per) of the bisection order, so neighbouring domains share
// that XCD's L2.  G8 blocks per XCD.  Returns -1 past the range.
__device__ inline int domain_of(const SweepArgs& a, int b, int k, int G8) {
  const int x = b % 8, i = b / 8;
  const int local = i + k * G8;
  if (local >= a.per_xcd) return -1;
  const int d = x * a.per_xcd + local;
  return d < a.P ? d : -1;
}

// Accumulate the previous sweep's contact forces on one particle entry, in
// ascending contact id: acc -= F (body 1) or += F (body 2), tacc -= r q.
template <int DIM>
__device__ inline void add_record(const double* rin, int ent, double rp,
                                  double* acc, double* tacc) {
  if (DIM == 2) {
    const double4 r4 = *(const double4*)(rin + (int64_t)(ent >> 1) * cd_rec(2));
    acc[0] = (ent & 1) ? acc[0] + r4.z : acc[0] - r4.z;
    acc[1] = (ent & 1) ? acc[1] + r4.w : acc[1] - r4.w;
    tacc[0] = tacc[0] - rp * r4.y;
  } else {
    double F[3], Q[3];
    cd_record_force3(rin, ent >> 1, F, Q);
    for (int k = 0; k < 3; ++k) acc[k] = (ent & 1) ? acc[k] + F[k] : acc[k] - F[k];
    for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * Q[k];
  }
}

template <int DIM>
__device__ inline void gather_forces(const SweepArgs& a, const double* rin, int64_t e, int4 r4i,
                                     double rp, double* acc, double* tacc) {
  constexpr int REC = cd_rec(DIM);
  constexpr int KW = DIM == 2 ? 8 : 16;
  // incidence rows: KW/4 planes of int4 (plane q: entries 4q..4q+3); the
  // first plane (r4i) is read by the caller
  const int4* rows = (const int4*)a.drow;
  const int64_t E = a.dpe;
  if (r4i.x == -2) {
    // more incidences than a row holds: the pointer list
    const int e1 = a.dinc_ptr[e + 1];
    for (int x = a.dinc_ptr[e]; x < e1; ++x) add_record<DIM>(rin, a.dinc[x], rp, acc, tacc);
    return;
  }
  // valid entries come first; the next plane is read only after a full one
  for (int q = 0; q < KW / 4; ++q) {
    const int ent[4] = {r4i.x, r4i.y, r4i.z, r4i.w};
    if (DIM == 2) {
      double4 rec[4];
      for (int u = 0; u < 4; ++u)
        if (ent[u] >= 0) rec[u] = *(const double4*)(rin + (int64_t)(ent[u] >> 1) * REC);
      for (int u = 0; u < 4; ++u) {
        if (ent[u] < 0) break;
        acc[0] = (ent[u] & 1) ? acc[0] + rec[u].z : acc[0] - rec[u].z;
        acc[1] = (ent[u] & 1) ? acc[1] + rec[u].w : acc[1] - rec[u].w;
        tacc[0] = tacc[0] - rp * rec[u].y;
      }
    } else {
      double F[4][3], Q[4][3];
      for (int u = 0; u < 4; ++u)
        if (ent[u] >= 0) cd_record_force3(rin, ent[u] >> 1, F[u], Q[u]);
      for (int u = 0; u < 4; ++u) {
        if (ent[u] < 0) break;
        for (int k = 0; k < 3; ++k) acc[k] = (ent[u] & 1) ? acc[k] + F[u][k] : acc[k] - F[u][k];
        for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * Q[u][k];
      }
    }
    if (ent[3] < 0 || q + 1 == KW / 4) break;
    r4i = rows[(q + 1) * E + e];
  }
}

// Static data of one contact, read from memory into registers: body pair,
// frame, g_e/dt, dt w_n, dt w_t, their reciprocals (RECIP) and the previous
// force.
template <int DIM>
struct SlotPre {
  int2 ab;
  double f[Layout<DIM>::NG];
  double gdt, dwn, dwt, kn, kt;
  double mu;            // friction coefficient of the contact
  double Ro[DIM];
};

template <int DIM, bool RECIP>
__device__ inline void fetch_slot(const SweepArgs& a, const double* rin, int64_t s, SlotPre<DIM>& o) {
  constexpr int NG = Layout<DIM>::NG, REC = Layout<DIM>::REC;
  const int64_t cap = a.cap;
  const double* g = a.geo;
  o.ab = a.ab[s];
  if (DIM == 3 && !RECIP) {
    // staged 3D slots: the normal from the record block (the same cache
    // line as the force); the tangents follow from it (cd_tangents, the
    // operations of the domain build), 48 bytes per slot not read
    const double4 n4 = *(const double4*)(rin + s * REC + 4);
    o.f[0] = n4.x;
    o.f[1] = n4.y;
    o.f[2] = n4.z;
    if (NG == 9) cd_tangents(o.f);
  } else {
    for (int q = 0; q < NG; ++q) o.f[q] = g[q * cap + s];
  }
  o.gdt = g[G_GDT * cap + s];
  o.dwn = g[G_DWN * cap + s];
  o.dwt = g[G_DWT * cap + s];
  if (RECIP) {
    o.kn = g[G_KN * cap + s];
    o.kt = g[G_KT * cap + s];
  }
  // always a global load (the shared coefficient sits in device memory too):
  // choosing between device memory and the kernel arguments would compile to
  // a flat load, which waits for every outstanding load and store of the wave
  o.mu = a.mu_slot[s * a.mu_step];
  const double* ri = rin + s * REC;
  if (DIM == 2) {
    const double2 r2 = *(const double2*)ri;
    o.Ro[0] = r2.x;
    o.Ro[1] = r2.y;
  } else {
    const double4 r4 = *(const double4*)ri;   // the whole 32-byte record
    o.Ro[0] = r4.x;
    o.Ro[1] = r4.y;
    o.Ro[DIM - 1] = r4.z;
  }
}

// Marks a read-ahead register set as arrived on every path (also in waves
// with no contact to update): the empty statement reads every register, so
// the wait for exactly this set's loads is taken here and its registers can
// be reused later without draining all outstanding memory accesses.
template <int DIM>
__device__ inline void settle(const SlotPre<DIM>& c) {
  asm volatile("" ::"v"(c.ab.x), "v"(c.ab.y), "v"(c.f[0]), "v"(c.f[1]), "v"(c.gdt), "v"(c.dwn),
               "v"(c.dwt), "v"(c.kn), "v"(c.kt), "v"(c.mu), "v"(c.Ro[0]), "v"(c.Ro[1]));
  if (DIM == 3)
    asm volatile("" ::"v"(c.f[Layout<DIM>::NG - 1]), "v"(c.Ro[DIM - 1]));
}

// A body's staged record: velocities, dt/m, dt/I, r.
template <int DIM>
struct Body {
  double V[3], W[3], dm, di, r;
};

template <int DIM>
__device__ inline void read_body(const double* sp, int l, Body<DIM>& b) {
  const double2* p = (const double2*)(sp + (int64_t)Layout<DIM>::PS * l);
  if (DIM == 2) {
    const double2 x0 = p[0], x1 = p[1], x2 = p[2];
    b.V[0] = x0.x;
    b.V[1] = x0.y;
    b.W[0] = x1.x;
    b.dm = x1.y;
    b.di = x2.x;
    b.r = x2.y;
    b.V[2] = b.W[1] = b.W[2] = 0.0;
  } else {
    const double2 x0 = p[0], x1 = p[1], x2 = p[2], x3 = p[3], x4 = p[4];
    b.V[0] = x0.x;
    b.V[1] = x0.y;
    b.V[2] = x1.x;
    b.W[0] = x1.y;
    b.W[1] = x2.x;
    b.W[2] = x2.y;
    b.dm = x3.x;
    b.di = x3.y;
    b.r = x4.x;
  }
}

template <int DIM>
__device__ inline void write_velocities(double* sp, int l, const double* V, const double* W) {
  double2* p = (double2*)(sp + (int64_t)Layout<DIM>::PS * l);
  if (DIM == 2) {
    p[0] = make_double2(V[0], V[1]);
    sp[(int64_t)Layout<DIM>::PS * l + 2] = W[0];
  } else {
    p[0] = make_double2(V[0], V[1]);
    p[1] = make_double2(V[2], W[0]);
    p[2] = make_double2(W[1], W[2]);
  }
}

// Convergence test values of one contact (Sec. 2.1): |R_new - R_old|^2
// against alpha |R_new + R_old|^2, and |R_new| for R_avg.
template <int DIM>
__device__ inline void account(const double* Rold, const double* Rn, double alpha,
                               long long& npass, double& maxd, double& sumr) {
  double d2 = 0.0, s2 = 0.0, qq = 0.0;
  for (int q = 0; q < DIM; ++q) {
    double a1 = Rn[q], a0 = Rold[q];
    d2 = d2 + (a1 - a0) * (a1 - a0);
    s2 = s2 + (a1 + a0) * (a1 + a0);
    qq = qq + a1 * a1;
  }
  sumr += sqrt(qq);
  if (d2 < alpha * s2 || d2 == 0.0) npass += 1;
  else if (d2 > maxd || d2 != d2) maxd = d2;
}

// The force law for one contact with the current velocities of its bodies
// (staged particle records at sp; body 2 < 0 is wall -1-b with velocity
// wu), the change applied to both bodies, the new record written to `ro`,
// and the contact's test values accounted.  APPLY = false (a contact
// updated in parallel, Sec. 2.3): the change is not applied to the bodies,
// which see it only through the next exchange.
// MOBILE: walls may have finite mass (wm: dt/M per wall, 0 for a wall of
// prescribed motion); such a wall's domain copy of its velocity in `wu` takes
// the normal part of the change, (dt/M) dR_n n (n = -nu).
template <int DIM, bool APPLY = true, bool MOBILE = false>
__device__ inline void update_contact(double* sp, double* wu, const SlotPre<DIM>& c,
                                      double alpha, double* ro, long long& npass,
                                      double& maxd, double& sumr, const double* wm = nullptr) {
  constexpr int DR = Layout<DIM>::DR;
  const int la = c.ab.x, lb = c.ab.y;
  Body<DIM> A, B;
  read_body<DIM>(sp, la, A);
  if (lb >= 0) {
    read_body<DIM>(sp, lb, B);
  } else {
    for (int q = 0; q < 3; ++q) B.V[q] = B.W[q] = 0.0;
    for (int q = 0; q < DIM; ++q) B.V[q] = wu[(-1 - lb) * DIM + q];
    B.dm = B.di = B.r = 0.0;
  }
  double nv[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < DIM; ++q) nv[q] = c.f[q];
  if (DIM == 2) {
    t1[0] = -nv[1];
    t1[1] = nv[0];
  } else {
    for (int q = 0; q < 3; ++q) {
      t1[q] = c.f[3 + q];
      t2[q] = c.f[6 + q];
    }
  }
  double Rold[3] = {0.0, 0.0, 0.0}, dwR[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < DIM; ++q) Rold[q] = c.Ro[q];
  dwR[0] = c.dwn * Rold[0];
  for (int q = 1; q < DIM; ++q) dwR[q] = c.dwt * Rold[q];
  double Rn[3] = {0.0, 0.0, 0.0};
  local_force<DIM>(nv, t1, t2, c.gdt, dwR, c.kn, c.kt, c.mu, A.r, B.r, A.V, A.W, B.V, B.W, Rn);
  const double dRn = Rn[0] - Rold[0], dR1 = Rn[1] - Rold[1];
  const double dR2 = DIM == 3 ? Rn[2] - Rold[2] : 0.0;
  double dF[3], dq[3];
  for (int q = 0; q < DIM; ++q) {
    dF[q] = dRn * nv[q] + dR1 * t1[q];
    if (DIM == 3) dF[q] = dF[q] + dR2 * t2[q];
  }
  if (DIM == 2) {
    dq[0] = dR1;
  } else {
    for (int q = 0; q < 3; ++q) dq[q] = dR1 * t2[q] - dR2 * t1[q];
  }
  double Va[3], Wa[3];
  for (int q = 0; q < DIM; ++q) Va[q] = A.V[q] - A.dm * dF[q];
  for (int q = 0; q < DR; ++q) Wa[q] = A.W[q] - A.di * (A.r * dq[q]);
  if (APPLY) write_velocities<DIM>(sp, la, Va, Wa);
  if (APPLY && lb >= 0) {
    double Vb[3], Wb[3];
    for (int q = 0; q < DIM; ++q) Vb[q] = B.V[q] + B.dm * dF[q];
    for (int q = 0; q < DR; ++q) Wb[q] = B.W[q] - B.di * (B.r * dq[q]);
    write_velocities<DIM>(sp, lb, Vb, Wb);
  } else if (MOBILE && APPLY) {
    const int w = -1 - lb;
    const double dtim = wm[w];
    if (dtim != 0.0)
      for (int q = 0; q < DIM; ++q) wu[w * DIM + q] = B.V[q] + dtim * (dRn * nv[q]);
  }
  // new record: frame force, world force, torque per unit lever (streamed
  // out: nothing in this launch reads it back)
  if (DIM == 2) {
    const nt4 v4 = {Rn[0], Rn[1], Rn[0] * nv[0] + Rn[1] * t1[0], Rn[0] * nv[1] + Rn[1] * t1[1]};
    __builtin_nontemporal_store(v4, (nt4*)ro);
  } else {
    // the frame force only: readers rebuild F and n x R from it and the normal
    const nt4 v0 = {Rn[0], Rn[1], Rn[2], 0.0};
    __builtin_nontemporal_store(v0, (nt4*)ro);
  }
  account<DIM>(Rold, Rn, alpha, npass, maxd, sumr);
}

// Base data of one domain particle entry read into registers: base
// velocities, external force and torque, dt/m, dt/I, r, and the first plane
// of its incidence row.
template <int DIM>
struct EntryPre {
  double v[DIM], w[Layout<DIM>::DR], f[DIM], t[Layout<DIM>::DR], dm, di, r;
  int4 row;
  int4 row1;   // the second plane when the first is full (staged form only)
  int hb;      // list index of the first foreign incidence (staged form only)
};

// The entry's external force and torque.  Forces and torques are flagged
// apart (gravity comes without torques): a part that is +0.0 on every body
// is set to +0.0 without reading, the same value the read would give.
template <int DIM>
__device__ inline void entry_ext(const SweepArgs& a, int64_t e, EntryPre<DIM>& o) {
  constexpr int DR = Layout<DIM>::DR;
  const int64_t E = a.dpe;
  const int q = DIM + DR;
  if (a.ext_zero & 1) {
    for (int k = 0; k < DIM; ++k) o.f[k] = 0.0;
  } else {
    for (int k = 0; k < DIM; ++k) o.f[k] = a.dpb[(q + k) * E + e];
  }
  if (a.ext_zero & 2) {
    for (int k = 0; k < DR; ++k) o.t[k] = 0.0;
  } else {
    for (int k = 0; k < DR; ++k) o.t[k] = a.dpb[(q + DIM + k) * E + e];
  }
}

// EXT = false: the external force and torque are left for entry_ext (read
// later, so that they do not occupy registers while the rest is in flight).
template <int DIM, bool EXT = true>
__device__ inline void entry_load(const SweepArgs& a, int64_t e, EntryPre<DIM>& o) {
  constexpr int DR = Layout<DIM>::DR;
  const int64_t E = a.dpe;
  for (int k = 0; k < DIM; ++k) o.v[k] = a.dpb[k * E + e];
  for (int k = 0; k < DR; ++k) o.w[k] = a.dpb[(DIM + k) * E + e];
  int q = DIM + DR;
  if (EXT) entry_ext<DIM>(a, e, o);
  q += DIM + DR;
  o.dm = a.dpb[q * E + e];
  o.di = a.dpb[(q + 1) * E + e];
  o.r = a.dpb[(q + 2) * E + e];
  o.row = ((const int4*)a.drow)[e];
  o.hb = a.hoff[e];
}

// The second row plane of an entry whose first plane is full (read once
// the first has arrived; most entries need only the first)
template <int DIM>
__device__ inline void entry_row1(const SweepArgs& a, int64_t e, EntryPre<DIM>& o) {
  o.row1 = make_int4(-1, -1, -1, -1);
  if (o.row.w >= 0) o.row1 = ((const int4*)a.drow)[a.dpe + e];
}

// The entry's velocities from its base data and the previous sweep's forces
// on it (ascending contact id), written as staged particle record l.
template <int DIM>
__device__ inline void entry_finish(const SweepArgs& a, const double* rin, int64_t e,
                                    const EntryPre<DIM>& o, double* sp, int l) {
  using L = Layout<DIM>;
  constexpr int DR = L::DR, PS = L::PS;
  double acc[DIM], tacc[DR];
  for (int k = 0; k < DIM; ++k) acc[k] = o.f[k];
  for (int k = 0; k < DR; ++k) tacc[k] = o.t[k];
  gather_forces<DIM>(a, rin, e, o.row, o.r, acc, tacc);
  double* pr = sp + (int64_t)PS * l;
  for (int k = 0; k < DIM; ++k) pr[k] = o.v[k] + o.dm * acc[k];
  for (int k = 0; k < DR; ++k) pr[L::P_W + k] = o.w[k] + o.di * tacc[k];
  pr[L::P_DM] = o.dm;
  pr[L::P_DI] = o.di;
  pr[L::P_R] = o.r;
}

// World force F and torque factor Q (2D: R_t; 3D: t2 R_1 - t1 R_2) of the
// domain's own slot k from its staged copy (the same products as the
// record's, so the same values)
template <int DIM>
__device__ inline void own_force(const double* sl, int nct, int k, double* F, double* Q) {
  constexpr int NG = Layout<DIM>::NG, NGS = Layout<DIM>::NGS;
  double f[NG], R[DIM];
  for (int q = 0; q < NGS; ++q) f[q] = sl[(1 + q) * nct + k];
  if (NG == 9) cd_tangents(f);
  for (int q = 0; q < DIM; ++q) R[q] = sl[(4 + NGS + q) * nct + k];
  if (DIM == 2) {
    const double t0 = -f[1], t1 = f[0];
    F[0] = R[0] * f[0] + R[1] * t0;
    F[1] = R[0] * f[1] + R[1] * t1;
    Q[0] = R[1];
  } else {
    for (int q = 0; q < 3; ++q) {
      const double fk = R[0] * f[q] + R[1] * f[3 + q];
      F[q] = fk + R[2] * f[6 + q];
      Q[q] = R[1] * f[6 + q] - R[2] * f[3 + q];
    }
  }
}

// F and Q of the previous sweep's force of slot s: from the staged copy when the slot
// is one of the domain's own (the same products as the record's, so the
// same values), else from the record.
template <int DIM>
__device__ inline void incidence_force(const double* rin, const double* sl,
                                       int cs, int nct, int64_t s, double* F, double* Q) {
  constexpr int REC = Layout<DIM>::REC;
  const int64_t k = s - cs;
  if (k >= 0 && k < nct) {
    own_force<DIM>(sl, nct, (int)k, F, Q);
  } else if (DIM == 2) {
    const double4 r4 = *(const double4*)(rin + s * REC);
    F[0] = r4.z;
    F[1] = r4.w;
    Q[0] = r4.y;
  } else {
    cd_record_force3(rin, s, F, Q);
  }
}

// gather_forces with the domain's own contacts read from its staged copy
template <int DIM>
__device__ inline void gather_forces_staged(const SweepArgs& a, const double* rin, int64_t e,
                                            int4 r4i, double rp, const double* sl, int cs,
                                            int nct, double* acc, double* tacc) {
  constexpr int DR = Layout<DIM>::DR;
  constexpr int KW = DIM == 2 ? 8 : 16;
  const int4* rows = (const int4*)a.drow;
  const int64_t E = a.dpe;
  auto add = [&](int ent, const double* F, const double* Q) {
    for (int k = 0; k < DIM; ++k) acc[k] = (ent & 1) ? acc[k] + F[k] : acc[k] - F[k];
    for (int k = 0; k < DR; ++k) tacc[k] = tacc[k] - rp * Q[k];
  };
  if (r4i.x == -2) {
    const int e1 = a.dinc_ptr[e + 1];
    for (int x = a.dinc_ptr[e]; x < e1; ++x) {
      const int ent = a.dinc[x];
      double F[DIM], Q[DR];
      incidence_force<DIM>(rin, sl, cs, nct, ent >> 1, F, Q);
      add(ent, F, Q);
    }
    return;
  }
  for (int q = 0; q < KW / 4; ++q) {
    const int ent[4] = {r4i.x, r4i.y, r4i.z, r4i.w};
    double F[4][DIM], Q[4][DR];
    for (int u = 0; u < 4; ++u)
      if (ent[u] >= 0) incidence_force<DIM>(rin, sl, cs, nct, ent[u] >> 1, F[u], Q[u]);
    for (int u = 0; u < 4; ++u) {
      if (ent[u] < 0) break;
      add(ent[u], F[u], Q[u]);
    }
    if (ent[3] < 0 || q + 1 == KW / 4) break;
    r4i = rows[(q + 1) * E + e];
  }
}

// entry_finish with the domain's own contacts read from its staged copy
template <int DIM>
__device__ inline void entry_finish_staged(const SweepArgs& a, const double* rin, int64_t e,
                                           const EntryPre<DIM>& o, double* sp, int l,
                                           const double* sl, int cs, int nct) {
  using L = Layout<DIM>;
  constexpr int DR = L::DR, PS = L::PS;
  double acc[DIM], tacc[DR];
  for (int k = 0; k < DIM; ++k) acc[k] = o.f[k];
  for (int k = 0; k < DR; ++k) tacc[k] = o.t[k];
  gather_forces_staged<DIM>(a, rin, e, o.row, o.r, sl, cs, nct, acc, tacc);
  double* pr = sp + (int64_t)PS * l;
  for (int k = 0; k < DIM; ++k) pr[k] = o.v[k] + o.dm * acc[k];
  for (int k = 0; k < DR; ++k) pr[L::P_W + k] = o.w[k] + o.di * tacc[k];
  pr[L::P_DM] = o.dm;
  pr[L::P_DI] = o.di;
  pr[L::P_R] = o.r;
}

// The previous sweep's force of foreign slot s in registers (2D: the whole
// record; 3D: the frame force and the normal), issued before it is needed
template <int DIM>
struct HaloPre {
  double4 r4, n4;
};

template <int DIM>
__device__ inline void halo_load(const double* rin, int64_t s, HaloPre<DIM>& o) {
  o.r4 = *(const double4*)(rin + s * cd_rec(DIM));
  if (DIM == 3) o.n4 = *(const double4*)(rin + s * cd_rec(DIM) + 4);
}

// Stores F and Q of a foreign incidence as item h of the domain's LDS block
// of nh items (column q at q nh): the values add_record computes from the
// record.
template <int DIM>
__device__ inline void halo_put(const HaloPre<DIM>& o, double* hl, int nh, int h) {
  if (DIM == 2) {
    hl[h] = o.r4.z;
    hl[nh + h] = o.r4.w;
    hl[2 * nh + h] = o.r4.y;
  } else {
    double f[9] = {o.n4.x, o.n4.y, o.n4.z, 0, 0, 0, 0, 0, 0};
    cd_tangents(f);
    for (int q = 0; q < 3; ++q) {
      const double fk = o.r4.x * f[q] + o.r4.y * f[3 + q];
      hl[q * nh + h] = fk + o.r4.z * f[6 + q];
      hl[(3 + q) * nh + h] = o.r4.y * f[6 + q] - o.r4.z * f[3 + q];
    }
  }
}

// The exchange of one particle entry entirely from LDS: its incidences in
// row order (ascending contact id), the domain's own from the staged slots,
// foreign ones as the next item of the entry's run in the staged block hl
// (items hb - hs on).
template <int DIM>
__device__ inline void gather_lds(const SweepArgs& a, int64_t e, const EntryPre<DIM>& o,
                                  const double* sl, int cs, int nct, const double* hl, int nh,
                                  int hs, double* acc, double* tacc) {
  constexpr int DR = Layout<DIM>::DR;
  constexpr int KW = DIM == 2 ? 8 : 16;
  int hk = o.hb - hs;
  const double rp = o.r;
  auto one = [&](int ent) {
    const int k = (ent >> 1) - cs;
    double F[DIM], Q[DR];
    if (k >= 0 && k < nct) {
      own_force<DIM>(sl, nct, k, F, Q);
    } else {
      for (int q = 0; q < DIM; ++q) F[q] = hl[q * nh + hk];
      for (int q = 0; q < DR; ++q) Q[q] = hl[(DIM + q) * nh + hk];
      ++hk;
    }
    for (int q = 0; q < DIM; ++q) acc[q] = (ent & 1) ? acc[q] + F[q] : acc[q] - F[q];
    for (int q = 0; q < DR; ++q) tacc[q] = tacc[q] - rp * Q[q];
  };
  if (o.row.x == -2) {
    // more incidences than a row holds: the pointer list
    const int e1 = a.dinc_ptr[e + 1];
    for (int x = a.dinc_ptr[e]; x < e1; ++x) one(a.dinc[x]);
    return;
  }
  const int4* rows = (const int4*)a.drow;
  int4 r = o.row;
  for (int q = 0; q < KW / 4; ++q) {
    if (q == 1) r = o.row1;
    else if (q > 1) r = rows[q * a.dpe + e];
    if (r.x < 0) break;
    one(r.x);
    if (r.y < 0) break;
    one(r.y);
    if (r.z < 0) break;
    one(r.z);
    if (r.w < 0) break;
    one(r.w);
  }
}

// The entry's staged record from its base data and the summed forces
template <int DIM>
__device__ inline void entry_write(const EntryPre<DIM>& o, const double* acc, const double* tacc,
                                   double* sp, int l) {
  using L = Layout<DIM>;
  constexpr int DR = L::DR, PS = L::PS;
  double* pr = sp + (int64_t)PS * l;
  for (int k = 0; k < DIM; ++k) pr[k] = o.v[k] + o.dm * acc[k];
  for (int k = 0; k < DR; ++k) pr[L::P_W + k] = o.w[k] + o.di * tacc[k];
  pr[L::P_DM] = o.dm;
  pr[L::P_DI] = o.di;
  pr[L::P_R] = o.r;
}

// entry_finish with the exchange from LDS (gather_lds)
template <int DIM>
__device__ inline void entry_finish_lds(const SweepArgs& a, int64_t e, const EntryPre<DIM>& o,
                                        double* sp, int l, const double* sl, int cs, int nct,
                                        const double* hl, int nh, int hs) {
  constexpr int DR = Layout<DIM>::DR;
  double acc[DIM], tacc[DR];
  for (int k = 0; k < DIM; ++k) acc[k] = o.f[k];
  for (int k = 0; k < DR; ++k) tacc[k] = o.t[k];
  gather_lds<DIM>(a, e, o, sl, cs, nct, hl, nh, hs, acc, tacc);
  entry_write<DIM>(o, acc, tacc, sp, l);
}

// Per-domain values a workgroup needs before its sweep: the descriptor
// (first slot, slots, first particle entry, entries, colours, largest
// colour), one colour
// offset and one wall velocity component per thread.  Read before the stop
// check so that their latency overlaps it.
struct DomainHead {
  int cs, nct, ps, np, ncol;
  int widest;   // contacts of the domain's largest colour
  int wmask;    // walls of finite mass the domain touches (bit w)
  int hs, nh;   // the domain's foreign incidences: first list index, count
  int co;       // colour offset number threadIdx.x (threads 0..CD_MAX_COLORS)
  double wu;    // wall velocity component number threadIdx.x
  int hsl;      // HSL: slot of foreign incidence number threadIdx.x (when
                // threadIdx.x < hstride; meaningful below the count nh)
};

// HSL: the domain's first foreign incidence slots too, so that their records
// can be requested as soon as the head has arrived.
template <int DIM, bool HSL = false>
__device__ inline DomainHead load_head(const SweepArgs& a, int d) {
  DomainHead h;
  const int* dd = a.ddesc + 8 * (int64_t)d;
  h.cs = dd[0];
  h.nct = dd[1];
  h.ps = dd[2];
  h.np = dd[3];
  h.ncol = dd[4];
  h.widest = dd[5];
  h.wmask = dd[6];
  const int2 hh = a.dhalo[d];
  h.hs = hh.x;
  h.nh = hh.y;
  const int tid = threadIdx.x;
  // every colour offset of a domain is written (unused ones hold the count)
  h.co = tid <= CD_MAX_COLORS ? a.dcol[(int64_t)d * (CD_MAX_COLORS + 1) + tid] : 0;
  h.wu = tid < a.n_walls * DIM ? a.walls_u[tid] : 0.0;
  h.hsl = HSL && tid < a.hstride ? a.hpad[(int64_t)d * a.hstride + tid] : 0;
  return h;
}

// Doubles per staged slot in LDS: body pair, frame, g_e/dt, dt w_n, dt w_t,
// previous force, and the friction coefficient when it is per slot.
template <int DIM>
__host__ __device__ constexpr int slot_stage_doubles(bool mu_per_slot) {
  static_assert(cd_stage_slot(DIM, false) == 1 + Layout<DIM>::NGS + 3 + DIM, "slot staging");
  return cd_stage_slot(DIM, mu_per_slot);
}

// The domain's contact data, slot k at column k of an LDS block of `nct`
// columns: pair (as one 8-byte word), frame, g_e/dt, dt w_n, dt w_t, the
// previous sweep's force, friction if per slot.
template <int DIM>
__device__ inline void put_slot(double* sl, int nct, int k, const SlotPre<DIM>& c, bool mu_slot) {
  constexpr int NG = Layout<DIM>::NGS;   // the normal only: 3D tangents are recomputed
  ((int2*)sl)[k] = c.ab;
  for (int q = 0; q < NG; ++q) sl[(1 + q) * nct + k] = c.f[q];
  sl[(1 + NG) * nct + k] = c.gdt;
  sl[(2 + NG) * nct + k] = c.dwn;
  sl[(3 + NG) * nct + k] = c.dwt;
  for (int q = 0; q < DIM; ++q) sl[(4 + NG + q) * nct + k] = c.Ro[q];
  if (mu_slot) sl[(4 + NG + DIM) * nct + k] = c.mu;
}

// Reads a staged slot back; the reciprocals 1/(dt w) are recomputed (the
// same IEEE division as when the slot constants were built).
template <int DIM>
__device__ inline void get_slot(const double* sl, int nct, int k, double mu0, bool mu_slot,
                                SlotPre<DIM>& c) {
  constexpr int NG = Layout<DIM>::NGS;
  c.ab = ((const int2*)sl)[k];
  for (int q = 0; q < NG; ++q) c.f[q] = sl[(1 + q) * nct + k];
  if (Layout<DIM>::NG == 9) cd_tangents(c.f);
  c.gdt = sl[(1 + NG) * nct + k];
  c.dwn = sl[(2 + NG) * nct + k];
  c.dwt = sl[(3 + NG) * nct + k];
  for (int q = 0; q < DIM; ++q) c.Ro[q] = sl[(4 + NG + q) * nct + k];
  c.mu = mu_slot ? sl[(4 + NG + DIM) * nct + k] : mu0;
  c.kn = 1.0 / c.dwn;
  c.kt = 1.0 / c.dwt;
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the finaliser applied to
// x plus the golden gamma.
__host__ __device__ inline unsigned long long rand_mix(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One sweep of domain d (head h) by the calling workgroup: exchange, then
// the colour-major update; accumulates the convergence test values of its
// contacts.  RAND: the random sequential order (Sec. 2.1) instead of the
// colours: slot s draws rand_mix(jkey ^ s), jkey = rand_mix(K ^ j) of sweep
// j, and thread 0 updates the domain's contacts one at a time by increasing
// draw (equal draws by slot); the draws and the ranked slots take 16 bytes
// of LDS per contact after the form's own staging.  GLOB: the particle
// records live in global scratch (domains too large for LDS).  STAGE: the
// domain's contact data and the previous sweep's forces of its foreign
// incidences are copied to LDS (all their loads in flight at once), the
// exchange reads only LDS and the colours read the contact data from
// there (HALO; without it the foreign forces are read from memory in the
// exchange, which needs less LDS); otherwise the exchange reads the records
// from memory and each thread reads its contact of the next colour into
// registers one colour ahead.
// MOBILE: walls of finite mass (Sec. 4.1): a domain touching one takes its
// velocity after the exchange from all its contacts' forces of the previous
// sweep (read in parallel into s_wtmp, summed in ascending contact id by one
// thread: u_n + dt/M (F - sum R_n) along nu, tangential part kept) and keeps
// its own copy in s_wu, which the domain's contacts with it update (s_wm:
// dt/M per wall).
template <int DIM, bool GLOB, bool STAGE, bool MIXED = false, bool RAND = false,
          bool MOBILE = false, bool HALO = true, class Idle>
__device__ inline void sweep_domain(const SweepArgs& a, int d, const DomainHead& h,
                                    const double* rin, double* rout, double* lds, int* s_co,
                                    double* s_wu, long long& npass, double& maxd, double& sumr,
                                    unsigned long long jkey, Idle&& idle,
                                    double* s_wm = nullptr, double* s_wtmp = nullptr) {
  static_assert(!(GLOB && STAGE), "staged contact data needs the particles in LDS");
  using L = Layout<DIM>;
  constexpr int REC = L::REC, PS = L::PS;
  const int tid = threadIdx.x, nthr = a.block;
  const int cs = h.cs, nct = h.nct, ps = h.ps, np = h.np, ncol = h.ncol;
  // mixed update (Sec. 2.3): colour 0 holds the contacts updated in parallel
  // and the sequential colours start at c0
  const int c0 = MIXED ? 1 : 0;
  double* sp = GLOB ? a.gscr + (int64_t)PS * ps : lds;
  const int* dcol = a.dcol + (int64_t)d * (CD_MAX_COLORS + 1);
  // 0. colour offsets and wall velocities to LDS
  if (tid <= CD_MAX_COLORS) s_co[tid] = h.co;
  for (int q = tid + nthr; q <= CD_MAX_COLORS; q += nthr) s_co[q] = dcol[q];
  if (tid < a.n_walls * DIM) s_wu[tid] = h.wu;
  if (MOBILE) {
    if (tid < a.n_walls) s_wm[tid] = a.walls_dtim[tid];
    if (h.wmask) {
      __syncthreads();
      for (int w = 0; w < a.n_walls; ++w) {
        if (!((h.wmask >> w) & 1)) continue;
        const int cnt = a.wall_cnt[w];
        const int* ls = a.wall_slot + (int64_t)w * a.cap;
        double acc = a.walls_force[w];
        for (int base = 0; base < cnt; base += nthr) {
          const int k = base + tid;
          if (k < cnt) s_wtmp[tid] = rin[(int64_t)ls[k] * REC];
          __syncthreads();
          if (tid == 0) {
            const int m = cnt - base < nthr ? cnt - base : nthr;
            for (int e = 0; e < m; ++e) acc = acc - s_wtmp[e];
          }
          __syncthreads();
        }
        if (tid == 0) {
          const double* nu = a.walls_n + w * DIM;
          const double* u = a.walls_u + w * DIM;
          double un = 0.0;
          for (int k = 0; k < DIM; ++k) un = un + nu[k] * u[k];
          const double un1 = un + a.walls_dtim[w] * acc;
          for (int k = 0; k < DIM; ++k) s_wu[w * DIM + k] = (u[k] - un * nu[k]) + un1 * nu[k];
        }
      }
    }
  }
  SlotPre<DIM> cur;
  int kc = -1;
  // staged form with the foreign forces (HALO): when the domain's entries
  // take one pass of the workgroup, the foreign forces share the LDS of the
  // particle records (every thread gathers into registers and writes its
  // record after a barrier); otherwise they follow the slots
  const int nh = HALO ? h.nh : 0;
  const bool uni = HALO && np <= nthr && np <= kUnionMax;
  constexpr int HW = cd_stage_halo(DIM);
  const int64_t ua = (int64_t)PS * np > (int64_t)HW * nh ? (int64_t)PS * np : (int64_t)HW * nh;
  double* sl = lds + (uni ? ua : (int64_t)PS * np);
  const bool mu_slot = a.mu_step != 0;
  double* hl = uni ? lds : sl + (int64_t)slot_stage_doubles<DIM>(mu_slot) * nct;
  if (STAGE && HALO) {
    // 1. this thread's first contact, first particle entry (without its
    //    external force) and first foreign incidence: every read is issued
    //    before any is used (indices clamped to valid ones so that the loads
    //    are unconditional); the contact data goes to LDS while the foreign
    //    incidences' forces are read, and those go to LDS as well, so that
    //    the exchange below reads nothing from memory
    {
      const int64_t s0 = nct > 0 ? cs : 0;
      const int64_t e1 = np > 0 ? ps + (tid < np ? tid : 0) : 0;
      EntryPre<DIM> ep;
      // the foreign records first: their slots came with the head, so these
      // reads are not a round after the others
      HaloPre<DIM> hp;
      if (tid < nh) halo_load<DIM>(rin, tid < a.hstride ? h.hsl : a.halo[h.hs + tid], hp);
      {
        SlotPre<DIM> x;
        fetch_slot<DIM, false>(a, rin, s0 + (tid < nct ? tid : 0), x);
        entry_load<DIM, false>(a, e1, ep);
        if (tid < nct) put_slot<DIM>(sl, nct, tid, x, mu_slot);
      }
      entry_row1<DIM>(a, e1, ep);
      // the rest of the contacts (domains of more than one per thread)
      for (int k = tid + nthr; k < nct; k += nthr) {
        SlotPre<DIM> z;
        fetch_slot<DIM, false>(a, rin, cs + k, z);
        put_slot<DIM>(sl, nct, k, z, mu_slot);
      }
      entry_ext<DIM>(a, e1, ep);
      if (tid < nh) halo_put<DIM>(hp, hl, nh, tid);
      for (int q = tid + nthr; q < nh; q += nthr) {
        HaloPre<DIM> hq;
        halo_load<DIM>(rin, a.halo[h.hs + q], hq);
        halo_put<DIM>(hq, hl, nh, q);
      }
      __syncthreads();
      if (uni) {
        constexpr int DR = Layout<DIM>::DR;
        double acc[DIM], tacc[DR];
        for (int k = 0; k < DIM; ++k) acc[k] = ep.f[k];
        for (int k = 0; k < DR; ++k) tacc[k] = ep.t[k];
        if (tid < np) gather_lds<DIM>(a, e1, ep, sl, cs, nct, hl, nh, h.hs, acc, tacc);
        // every gather has read the foreign forces before the records
        // overwrite them
        __syncthreads();
        if (tid < np) entry_write<DIM>(ep, acc, tacc, sp, tid);
      } else if (tid < np) {
        entry_finish_lds<DIM>(a, e1, ep, sp, tid, sl, cs, nct, hl, nh, h.hs);
      }
    }
    for (int l = tid + nthr; l < np; l += nthr) {
      EntryPre<DIM> ep;
      entry_load<DIM>(a, ps + l, ep);
      entry_row1<DIM>(a, ps + l, ep);
      entry_finish_lds<DIM>(a, ps + l, ep, sp, l, sl, cs, nct, hl, nh, h.hs);
    }
  } else if (STAGE) {
    // 1. this thread's first two contacts and first particle entry: every
    //    read is issued before any is used (indices clamped to valid ones
    //    so that the loads are unconditional), then the contact data goes
    //    to LDS while the entry's force gathers are in flight
    {
      const int k1 = tid, k2 = tid + nthr;
      SlotPre<DIM> x, y;
      EntryPre<DIM> ep;
      const int64_t s0 = nct > 0 ? cs : 0;
      fetch_slot<DIM, false>(a, rin, s0 + (k1 < nct ? k1 : 0), x);
      fetch_slot<DIM, false>(a, rin, s0 + (k2 < nct ? k2 : 0), y);
      const int64_t e1 = np > 0 ? ps + (tid < np ? tid : 0) : 0;
      entry_load<DIM>(a, e1, ep);
      if (k1 < nct) put_slot<DIM>(sl, nct, k1, x, mu_slot);
      if (k2 < nct) put_slot<DIM>(sl, nct, k2, y, mu_slot);
      if (DIM == 2) {
        // 2D: the gathers read whole 32-byte records, the domain's own mostly
        // from cache right after this workgroup read them
        if (tid < np) entry_finish<DIM>(a, rin, e1, ep, sp, tid);
      }
      // the rest of the contacts (domains of more than two per thread)
      for (int k = tid + 2 * nthr; k < nct; k += nthr) {
        SlotPre<DIM> z;
        fetch_slot<DIM, false>(a, rin, cs + k, z);
        put_slot<DIM>(sl, nct, k, z, mu_slot);
      }
      if (DIM == 3) {
        // 3D: the gathers read the domain's own contacts (most of a
        // particle's incidences) from the staged copy, only foreign ones
        // from memory
        __syncthreads();
        if (tid < np) entry_finish_staged<DIM>(a, rin, e1, ep, sp, tid, sl, cs, nct);
      }
    }
    for (int l = tid + nthr; l < np; l += nthr) {
      EntryPre<DIM> ep;
      entry_load<DIM>(a, ps + l, ep);
      if (DIM == 2) entry_finish<DIM>(a, rin, ps + l, ep, sp, l);
      else entry_finish_staged<DIM>(a, rin, ps + l, ep, sp, l, sl, cs, nct);
    }
  } else {
    if (!RAND && ncol > c0) {
      // this thread's contact of the first sequential colour read ahead
      // (its latency overlaps the exchange); lanes without one read the
      // first slot
      const int b0 = dcol[c0];
      kc = b0 + tid < dcol[c0 + 1] ? b0 + tid : -1;
      fetch_slot<DIM, true>(a, rin, cs + (kc >= 0 ? kc : 0), cur);
    }
    // 1. exchange: velocities from the previous sweep's forces
    for (int l = tid; l < np; l += nthr) {
      EntryPre<DIM> ep;
      entry_load<DIM>(a, ps + l, ep);
      entry_finish<DIM>(a, rin, ps + l, ep, sp, l);
    }
  }
  __syncthreads();
  if (RAND) {
    unsigned long long* key =
        (unsigned long long*)(STAGE ? (uni ? sl + (int64_t)slot_stage_doubles<DIM>(mu_slot) * nct
                                           : hl + (int64_t)cd_stage_halo(DIM) * nh)
                                    : (GLOB ? lds : lds + (int64_t)PS * np));
    int* perm = (int*)(key + nct);
    for (int k = tid; k < nct; k += nthr) key[k] = rand_mix(jkey ^ (unsigned long long)(cs + k));
    __syncthreads();
    for (int k = tid; k < nct; k += nthr) {
      const unsigned long long kk = key[k];
      int rank = 0;
      for (int m = 0; m < nct; ++m) {
        const unsigned long long km = key[m];
        rank += (km < kk || (km == kk && m < k)) ? 1 : 0;
      }
      perm[rank] = k;
    }
    __syncthreads();
    if (tid == 0) {
      const double mu0 = mu_slot ? 0.0 : a.mu_slot[0];
      for (int q = 0; q < nct; ++q) {
        const int k = perm[q];
        SlotPre<DIM> c;
        if (STAGE) get_slot<DIM>(sl, nct, k, mu0, mu_slot, c);
        else fetch_slot<DIM, true>(a, rin, cs + k, c);
        update_contact<DIM, true, MOBILE>(sp, s_wu, c, a.alpha, rout + (int64_t)(cs + k) * REC, npass, maxd,
                            sumr, s_wm);
      }
    }
    idle();
    return;
  }
  if (STAGE) {
    const double mu0 = mu_slot ? 0.0 : a.mu_slot[0];
    if (MIXED) {
      // the parallel contacts, every thread, from the velocities of the
      // exchange; their reads precede the colours' writes
      for (int k = s_co[0] + tid; k < s_co[1]; k += nthr) {
        SlotPre<DIM> c;
        get_slot<DIM>(sl, nct, k, mu0, mu_slot, c);
        update_contact<DIM, false>(sp, s_wu, c, a.alpha, rout + (int64_t)(cs + k) * REC, npass,
                                   maxd, sumr);
      }
      lds_barrier();
    }
    // 2. colour-major sequential update from the staged contact data
    if (h.widest <= 64) {
      // every colour fits one wavefront: the first wavefront updates them
      // all, ordered by its own LDS accesses (a wavefront's LDS operations
      // complete in issue order), with no workgroup barrier per colour; the
      // other wavefronts are free for `idle`
      if (tid < 64) {
        for (int col = c0; col < ncol; ++col) {
          const int k = s_co[col] + tid;
          if (k < s_co[col + 1]) {
            SlotPre<DIM> c;
            get_slot<DIM>(sl, nct, k, mu0, mu_slot, c);
            update_contact<DIM, true, MOBILE>(sp, s_wu, c, a.alpha, rout + (int64_t)(cs + k) * REC, npass,
                                maxd, sumr, s_wm);
          }
          wave_lds_order();
        }
      } else {
        idle();
      }
      return;
    }
    for (int col = c0; col < ncol; ++col) {
      const int k0 = s_co[col], k1 = s_co[col + 1];
      for (int k = k0 + tid; k < k1; k += nthr) {
        SlotPre<DIM> c;
        get_slot<DIM>(sl, nct, k, mu0, mu_slot, c);
        update_contact<DIM, true, MOBILE>(sp, s_wu, c, a.alpha, rout + (int64_t)(cs + k) * REC, npass, maxd,
                            sumr, s_wm);
      }
      // the colour's velocity updates must be seen by the next colour; the
      // record stores stay in flight
      lds_barrier();
    }
    idle();
    return;
  }
  // 2. colour-major sequential update.  Each thread's contact of the next
  // colour is read into the other of two register sets while this colour is
  // updated (no copy between the sets, so nothing waits for the read-ahead
  // or the record stores before the next colour needs them).
  auto colour = [&](int col, const SlotPre<DIM>& use, int ku, SlotPre<DIM>& pre, int& kp) {
    const int k0 = s_co[col], k1 = s_co[col + 1];
    // lanes without a next contact (all lanes in the last colour) read the
    // domain's first slot: the loads are issued on every path, so the wait
    // for them counts exactly instead of draining every outstanding access
    kp = (col + 1 < ncol && k1 + tid < s_co[col + 2]) ? k1 + tid : -1;
    fetch_slot<DIM, true>(a, rin, cs + (kp >= 0 ? kp : 0), pre);
    settle<DIM>(use);
    if (ku >= 0)
      update_contact<DIM, true, MOBILE>(sp, s_wu, use, a.alpha, rout + (int64_t)(cs + ku) * REC, npass,
                          maxd, sumr, s_wm);
    // colours wider than the workgroup (rare); the path ends with all its
    // memory accesses complete, so that it leaves no pending store whose
    // registers the common path would have to wait for
    if (k1 - k0 > nthr) {
      for (int k = k0 + tid + nthr; k < k1; k += nthr) {
        SlotPre<DIM> sd;
        fetch_slot<DIM, true>(a, rin, cs + k, sd);
        update_contact<DIM, true, MOBILE>(sp, s_wu, sd, a.alpha, rout + (int64_t)(cs + k) * REC, npass,
                            maxd, sumr, s_wm);
      }
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
    }
    // the colour's velocity updates must be seen by the next colour; the
    // record stores and the read-ahead loads stay in flight
    if (GLOB) __syncthreads();
    else lds_barrier();
  };
  if (MIXED) {
    // the parallel contacts (Sec. 2.3), every thread, from the velocities of
    // the exchange; their reads precede the colours' writes
    for (int k = s_co[0] + tid; k < s_co[1]; k += nthr) {
      SlotPre<DIM> pc;
      fetch_slot<DIM, true>(a, rin, cs + k, pc);
      update_contact<DIM, false>(sp, s_wu, pc, a.alpha, rout + (int64_t)(cs + k) * REC, npass,
                                 maxd, sumr);
    }
    if (GLOB) __syncthreads();
    else lds_barrier();
  }
  SlotPre<DIM> other;
  int ko = -1;
  int col = c0;
  for (; col + 1 < ncol; col += 2) {
    colour(col, cur, kc, other, ko);
    colour(col + 1, other, ko, cur, kc);
  }
  if (col < ncol) colour(col, cur, kc, other, ko);
  idle();
}

}  // namespace
