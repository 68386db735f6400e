// HIP kernels (gfx950) for the decorated-particle cycle of arXiv 2605.21794, Section 5:
// deposit of the monopole + dipole load (eq. rhs-assembly), periodic P1 Poisson solve with
// the zero-mean gauge (eq. lin-sys), gather of E = -phi_h' and of the projected phi_h'',
// and the kick / drift sub-flows of eq. sw-evolution.
//
// Layout: particles are five structure-of-arrays streams; one workgroup owns one tile of
// consecutive particles of one instance, so every load and store is coalesced.  The load
// vector is accumulated into an LDS-private copy of the grid (float64 LDS atomics, or float32
// (hi, lo) two-sum pairs under a 64-bit compare-and-swap, or float32 atomics in the naive
// mode), and each tile adds its grid into one of the instance's spread global accumulator
// copies.  The fused step needs no grid-wide wait: the accumulators form a ring of three
// entries, and every workgroup of the next launch solves the field of the entry the previous
// launch filled (a few microseconds of LDS work that overlap its first particle loads), so
// one kernel per step advances every instance and the kernel boundary is the only barrier.
//
// Rounding: every kernel is compiled without floating-point contraction, and the float64
// particle arithmetic follows the same operation order as the plain CPU definition, so the
// float64 push is bitwise reproducible from the same inputs; only sums differ in order.

#include "vp_internal.h"

#include "vp_device.h"

namespace vpk {

// Deposit of the current state only (eq. rhs-assembly), added into ring entry `phase`.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_deposit(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int tile0,
                                                 int ppt, int phase) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double* sacc = smem + 2 * ng;
  stage<MODE, TPB>(d, smem, sacc, false, true);
  const VPG T* __restrict__ Qp = gp<T>(d.Q);
  const VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  if constexpr (MODE == kFP32) {
    const float ihf = (float)d.inv_h;
    float* fa = reinterpret_cast<float*>(sacc);
    VP_TILE_LOOP_BEGIN
    float q[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; b[u] = psp[idx[u]]; w[u] = psip[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const float x = q[u] * ihf;
      const int j = cell_of_f(x, ng);
      const float s = frac01_f(x, j);
      atomicAdd(fa + j, w[u] * (1.0f - s) + b[u] * ihf);
      atomicAdd(fa + ((j + 1) & (ng - 1)), w[u] * s - b[u] * ihf);
    }
    VP_TILE_LOOP_END
  } else {
    const double inv_h = d.inv_h;
    const bool p2 = d.order == 2;
    const VPG T* __restrict__ Mqqp = gp<T>(d.Mqq);  // k = 3 only
    VP_TILE_LOOP_BEGIN
    T q[4], b[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; b[u] = psp[idx[u]]; w[u] = psip[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double psi = w[u], psd = b[u];
      const double x = (double)q[u] * inv_h;
      const int j = cell_of(x, ng);
      const double s = frac01(x, j);
      if (p2 && d.k3) {
        deposit_p2<MODE, true, true>(sacc, ng, j, s, psi, psd, inv_h, (double)Mqqp[idx[u]]);
      } else if (p2) {
        deposit_p2<MODE, true>(sacc, ng, j, s, psi, psd, inv_h);
      } else {
        lds_add<MODE>(sacc, j, psi * (1.0 - s) + psd * inv_h);
        lds_add<MODE>(sacc, (j + 1) & (ng - 1), psi * s - psd * inv_h);
      }
    }
    VP_TILE_LOOP_END
  }
  __syncthreads();
  flush<MODE, TPB>(d, sacc, phase, tl.local % d.acc_copies);
}

// Kick by `kick` then drift by `drift` with the field arrays.  With use_pending, the kick of
// each instance is dt/2 when its half-kick is pending in phase `phase` and 0 otherwise, and
// drift is 0.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_gather_push(const InstDev* __restrict__ insts,
                                                     const Tile* __restrict__ tiles, int tile0,
                                                     int ppt, double kick_in, double drift_in,
                                                     int use_pending, int phase) {
  extern __shared__ double smem[];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  double kick = kick_in, drift = drift_in;
  if (use_pending) {
    kick = gp(d.scal)->pend[phase] ? 0.5 * d.dt : 0.0;
    drift = 0.0;
  }
  if (kick == 0.0 && drift == 0.0) return;  // uniform per workgroup: no barrier skipped
  stage<MODE, TPB>(d, smem, nullptr, true, false);
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const bool do_kick = kick != 0.0, do_drift = drift != 0.0;
  if constexpr (MODE == kFP32) {
    const float* fE = reinterpret_cast<const float*>(smem);
    const float* fG = fE + ng;
    const float Lf = (float)d.L, ihf = (float)d.inv_h, kf = (float)kick, df = (float)drift;
    VP_TILE_LOOP_BEGIN
    float q[4], p[4], a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      float Q = q[u], P = p[u], qs = a[u], ps = b[u];
      const float xq = Q * ihf;
      const int i = cell_of_f(xq, ng);
      float Ei, gi;
      if (!d.general) {
        Ei = fE[i];
        gi = fG[i];
      } else {
        double e, g, uu;
        general_field(d, fE, fG, i, (double)Q * d.inv_h, (double)Q, 0.0, 0.0, e, g, uu);
        Ei = (float)e;
        gi = (float)g;
      }
      P = P + kf * Ei;
      qs = qs + kf * ps * gi;
      float Qn = Q + df * P;
      if (Qn < 0.0f) Qn += Lf;
      if (Qn >= Lf) Qn -= Lf;
      ps = ps - df * qs;
      if (do_kick) { Pp[idx[u]] = P; qsp[idx[u]] = qs; }
      if (do_drift) { Qp[idx[u]] = Qn; psp[idx[u]] = ps; }
    }
    VP_TILE_LOOP_END
  } else {
    const double L = d.L, inv_h = d.inv_h;
    const bool k3 = d.k3;  // second moments (uniform per workgroup)
    VPG T* __restrict__ M0p = gp<T>(d.Mqq);
    VPG T* __restrict__ M1p = gp<T>(d.Mqp);
    VPG T* __restrict__ M2p = gp<T>(d.Mpp);
    VP_TILE_LOOP_BEGIN
    T q[4], p[4], a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (v[u]) { q[u] = Qp[idx[u]]; p[u] = Pp[idx[u]]; a[u] = qsp[idx[u]]; b[u] = psp[idx[u]]; }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double Q = q[u];
      double P = p[u], qs = a[u], ps = b[u];
      const double xq = Q * inv_h;
      const int i = cell_of(xq, ng);
      double Ei, gi;
      if (!d.general) {
        Ei = smem[i];
        gi = smem[ng + i];
        if (d.order == 2) Ei = Ei - d.h * gi * (frac01(xq, i) - 0.5);  // P2: linear field
      } else {
        double uu;
        general_field(d, smem, smem + ng, i, xq, (double)Q, 0.0, 0.0, Ei, gi, uu);
      }
      double Mqq = 0.0, Mqp = 0.0, Mpp = 0.0, g3 = 0.0, uk = 0.0;
      if (k3) {
        Mqq = M0p[idx[u]];
        Mqp = M1p[idx[u]];
        Mpp = M2p[idx[u]];
        k3_external(d, Q, Mqq, g3, uk);
      }
      P = P + kick * Ei;
      qs = qs + kick * ps * gi;
      if (k3) {
        qs = qs - (0.5 * kick) * Mqq * g3;
        moments_kick(kick, gi, Mqq, Mqp, Mpp);
      }
      double Qn = Q + drift * P;
      if (Qn < 0.0) Qn += L;
      if (Qn >= L) Qn -= L;
      ps = ps - drift * qs;
      if (k3) moments_drift(drift, Mqq, Mqp, Mpp);
      if (do_kick) { Pp[idx[u]] = (T)P; qsp[idx[u]] = (T)qs; }
      if (do_drift) { Qp[idx[u]] = (T)Qn; psp[idx[u]] = (T)ps; }
      if (k3) { M0p[idx[u]] = (T)Mqq; M1p[idx[u]] = (T)Mqp; M2p[idx[u]] = (T)Mpp; }
    }
    VP_TILE_LOOP_END
  }
}

// Kinetic diagnostics at the integer step without touching the state: a pending half-kick
// is applied to local copies only.
template <int MODE, int TPB>
__global__ __launch_bounds__(TPB) void k_diag(const InstDev* __restrict__ insts,
                                              const Tile* __restrict__ tiles, int tile0,
                                              int ppt, int phase) {
  extern __shared__ double smem[];
  __shared__ double red[TPB / 64];
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  stage<MODE, TPB>(d, smem, nullptr, true, false);
  const VPG T* __restrict__ Qp = gp<T>(d.Q);
  const VPG T* __restrict__ Pp = gp<T>(d.P);
  const VPG T* __restrict__ qsp = gp<T>(d.qs);
  const VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  const int pend = gp(d.scal)->pend[phase];
  double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
  if constexpr (MODE == kFP32) {
    const float* fE = reinterpret_cast<const float*>(smem);
    const float* fG = fE + ng;
    const float ihf = (float)d.inv_h, hf = 0.5f * (float)d.dt;
    VP_TILE_LOOP_BEGIN
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const float Q = Qp[idx[u]], psi = psip[idx[u]], ps = psp[idx[u]];
      float P = Pp[idx[u]], qs = qsp[idx[u]];
      const float xq = Q * ihf;
      const int i = cell_of_f(xq, ng);
      float Ei, gi;
      if (!d.general) {
        Ei = fE[i];
        gi = fG[i];
      } else {
        double e, g, uu;
        general_field(d, fE, fG, i, (double)Q * d.inv_h, (double)Q, (double)psi, (double)ps, e,
                      g, uu);
        Ei = (float)e;
        gi = (float)g;
        Us += uu;
      }
      if (pend) {
        P = P + hf * Ei;
        qs = qs + hf * ps * gi;
      }
      const double Pd = P, qd = qs, wd = psi;
      Ks += 0.5 * wd * Pd * Pd + qd * Pd;
      Ms += wd * Pd + qd;
      Cs += wd;
    }
    VP_TILE_LOOP_END
  } else {
    const double inv_h = d.inv_h, half = 0.5 * d.dt;
    const bool k3 = d.k3;  // second moments (uniform per workgroup)
    VP_TILE_LOOP_BEGIN
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!v[u]) continue;
      const double Q = Qp[idx[u]], psi = psip[idx[u]], ps = psp[idx[u]];
      double P = Pp[idx[u]], qs = qsp[idx[u]];
      const double xq = Q * inv_h;
      const int i = cell_of(xq, ng);
      double Ei, gi;
      if (!d.general) {
        Ei = smem[i];
        gi = smem[ng + i];
        if (d.order == 2) Ei = Ei - d.h * gi * (frac01(xq, i) - 0.5);  // P2: linear field
      } else {
        double uu;
        general_field(d, smem, smem + ng, i, xq, Q, psi, ps, Ei, gi, uu);
        Us += uu;
      }
      double Mqq = 0.0, Mqp = 0.0, Mpp = 0.0, g3 = 0.0;
      if (k3) {
        Mqq = gp<T>(d.Mqq)[idx[u]];
        Mqp = gp<T>(d.Mqp)[idx[u]];
        Mpp = gp<T>(d.Mpp)[idx[u]];
        k3_external(d, Q, Mqq, g3, Us);
      }
      if (pend) {
        P = P + half * Ei;
        qs = qs + half * ps * gi;
        if (k3) {
          qs = qs - (0.5 * half) * Mqq * g3;
          moments_kick(half, gi, Mqq, Mqp, Mpp);
        }
      }
      Ks += 0.5 * psi * P * P + qs * P;
      if (k3) Ks += 0.5 * Mpp;
      Ms += psi * P + qs;
      Cs += psi;
    }
    VP_TILE_LOOP_END
  }
  const double Kb = block_sum<TPB>(Ks, red);
  const double Mb = block_sum<TPB>(Ms, red);
  const double Cb = block_sum<TPB>(Cs, red);
  const double Ub = block_sum<TPB>(Us, red);
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    gadd(&sc->Kd, Kb);
    gadd(&sc->momd, Mb);
    gadd(&sc->chgd, Cb);
    gadd(&sc->Ud, Ub);
  }
}

// One workgroup per listed slot: solve the field of ring entry `phase` and write the field
// arrays and the field summary (materialise); when the instance's last pass was a fused
// step, also write that step's record (the next fused pass would write the same record).
template <int MODE>
__global__ __launch_bounds__(kSolveThreads) void k_solve(const InstDev* __restrict__ insts,
                                                         const int* __restrict__ slots,
                                                         int phase) {
  extern __shared__ double smem[];
  __shared__ double sred[kSolveRed];
  const InstDev& d = insts[slots[blockIdx.x]];
  const int ng = d.ng;
  const bool p2 = d.order == 2;
  double* fE = smem;
  double* fG = smem + ng;
  double* phi = smem + 2 * ng;
  double* bt = smem + 3 * ng;
  double* fft = smem + 4 * ng;
  // P2: b~ of vertices and midpoints, after the FFT scratch when this instance uses it
  double* p2b = smem + (d.solver == VP_SOLVE_FFT ? 7 : 4) * ng;
  SolveIn sin_;
  solve_load<MODE>(d, phase, true, sin_);
  double sum[7];
  solve_compute<kSolveThreads>(d, sin_, true, bt, fE, fG, sred, fft, phi, sum,
                               p2 ? p2b : nullptr);
  VPG double* bt_g = gp(d.bt);
  VPG double* E_g = gp(d.E);
  VPG double* g_g = gp(d.g);
  VPG double* Phi_g = gp(d.Phi);
  VPG float* Ef_g = gp(d.Ef);
  VPG float* gf_g = gp(d.gf);
  if (!p2) {
    for (int e = threadIdx.x; e < ng; e += kSolveThreads) {
      const double Ee = fE[e], ge = fG[e];
      bt_g[e] = bt[e];
      E_g[e] = Ee;
      Ef_g[e] = (float)Ee;
      g_g[e] = ge;
      gf_g[e] = (float)ge;
      Phi_g[e] = phi[e];
    }
  } else {
    // midpoint potentials from their own rows, Phi_m = (3h b~_m + 8 (Phi_e + Phi_{e+1})) / 16;
    // then the P2 gauge: shift by c so that (h/3) sum Phi_v + (2h/3) sum Phi_m = 0
    const int per = solve_per(ng);
    double pm[kSolvePer];
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
      pm[k] = 0.0;
      const int e = threadIdx.x * per + k;
      if (k < per && e < ng) {
        pm[k] = (3.0 * d.h * p2b[ng + e] + 8.0 * (phi[e] + phi[(e + 1) & (ng - 1)])) / 16.0;
        part += phi[e] + 2.0 * pm[k];
      }
    }
    const double c = -block_sum<kSolveThreads>(part, sred) / (3.0 * (double)ng);
#pragma unroll
    for (int k = 0; k < kSolvePer; ++k) {
      const int e = threadIdx.x * per + k;
      if (k < per && e < ng) {
        bt_g[e] = p2b[e];
        bt_g[ng + e] = p2b[ng + e];
        Phi_g[e] = phi[e] + c;
        Phi_g[ng + e] = pm[k] + c;
      }
    }
    for (int e = threadIdx.x; e < ng; e += kSolveThreads) {
      const double Ee = fE[e], ge = fG[e];
      E_g[e] = Ee;
      Ef_g[e] = (float)Ee;
      g_g[e] = ge;
      gf_g[e] = (float)ge;
    }
  }
  if (threadIdx.x == 0) {
    VPG InstScal* sc = gp(d.scal);
    const int r2 = ring_prev(phase);
    if (sc->pend[phase] && sc->step >= 1)
      write_record(d, sc->step - 1, sum[3], sum[4], sum[5], sum[6], sc->W[r2], sc->e1r[r2],
                   sc->e1i[r2]);
    sc->W[phase] = sum[0];
    sc->e1r[phase] = sum[1];
    sc->e1i[phase] = sum[2];
    if (!isfinite(sum[0])) sc->nonfinite = 1;
  }
}

// Ring maintenance, one workgroup per listed slot (see RingOp).
template <typename A>
__global__ __launch_bounds__(256) void k_ring(const InstDev* __restrict__ insts,
                                              const int* __restrict__ slots, int op, int phase) {
  const InstDev& d = insts[slots[blockIdx.x]];
  const int nacc = d.nacc;
  VPG A* acc = gp<A>(reinterpret_cast<A*>(d.acc));
  for (int j = threadIdx.x; j < nacc; j += 256) {
    if (op == kRingFold) {
      double s = 0.0;
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) s += (double)acc[acc_off(d, phase, c) + j];
      acc[acc_off(d, phase, 0) + j] = (A)s;
      for (int c = 1; c < VP_MAX_ACC_COPIES; ++c) acc[acc_off(d, phase, c) + j] = (A)0;
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) {
        acc[acc_off(d, ring_next(phase), c) + j] = (A)0;
        acc[acc_off(d, ring_prev(phase), c) + j] = (A)0;
      }
    } else {
      for (int c = 0; c < VP_MAX_ACC_COPIES; ++c) acc[acc_off(d, phase, c) + j] = (A)0;
    }
  }
  if (op == kRingFold) {
    // per-tile kinetic sums: the tile count may change, so each entry's sum moves to tile 0
    // and the other tiles are cleared.  Thread t adds tiles t, t + 256, ... in order, then
    // thread 0 adds the 256 partial sums in thread order (fixed order, deterministic).
    __shared__ double part[256];
    VPG double* kin = gp(d.kin);
    for (int rf = 0; rf < kRing * kKinFields; ++rf) {
      const int r = rf / kKinFields, f = rf % kKinFields;
      VPG double* base = kin + (size_t)r * d.kin_cap * kKinFields + f;
      double acc_t = 0.0;
      for (int t = threadIdx.x; t < d.kin_cap; t += 256) acc_t += base[(size_t)t * kKinFields];
      __syncthreads();
      part[threadIdx.x] = acc_t;
      __syncthreads();
      for (int t = threadIdx.x; t < d.kin_cap; t += 256) base[(size_t)t * kKinFields] = 0.0;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < 256; ++t) s += part[t];
        base[0] = s;
      }
    }
  }
}

__global__ void k_slot_scalars(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                               int nslots, int op, int phase) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  VPG InstScal* sc = gp(insts[slots[t]].scal);
  if (op == kScalClearDiag) {
    sc->Kd = 0.0;
    sc->Ud = 0.0;
    sc->momd = 0.0;
    sc->chgd = 0.0;
  } else if (op == kScalClearPending) {
    sc->pend[phase] = 0;
  } else if (op == kScalPersistStart) {
    sc->frozen = sc->nonfinite;
    for (int gr = 0; gr < kArriveGroups; ++gr) sc->arrive[gr * kArriveStride] = 0u;
    sc->top[0] = 0u;
    for (int f = 0; f < kReleaseFlags; ++f) sc->release[f * kArriveStride] = 0u;
  }
}

__global__ void k_slot_status(const InstDev* __restrict__ insts, const int* __restrict__ slots,
                              int nslots, long long* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  const VPG InstScal* sc = gp(insts[slots[t]].scal);
  out[2 * t] = sc->step;
  out[2 * t + 1] = sc->nonfinite;
}

// Zero n8 64-bit words, then a trailing 32-bit word when tail4 (an odd count of floats).
__global__ void k_fill_zero(unsigned long long* p, size_t n8, bool tail4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = t; i < n8; i += stride) p[i] = 0ull;
  if (tail4 && t == 0) reinterpret_cast<unsigned*>(p + n8)[0] = 0u;
}

template <typename T>
__global__ void k_cell_index(const InstDev* __restrict__ insts, int slot, int* __restrict__ cells,
                             long long n) {
  const InstDev& d = insts[slot];
  const VPG T* Qp = gp<T>(d.Q);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    cells[k] = cell_of((double)Qp[k] * d.inv_h, d.ng);
}

// ------------------------------------------------------------------ chunked stable sort
// Workgroup b sorts particles [b*chunk, min(n, (b+1)*chunk)) by cell (float64 index
// formula) with two stable 5-bit counting passes in LDS, then permutes the five arrays
// in place through an LDS staging buffer.
template <typename T>
__device__ void permute_array(VPG T* __restrict__ X, long long c0, int m, const unsigned short* order,
                              T* stagebuf) {
  for (int k = threadIdx.x; k < m; k += kBlock) stagebuf[k] = X[c0 + order[k]];
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += kBlock) X[c0 + k] = stagebuf[k];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sort(const InstDev* __restrict__ insts, int slot,
                                                 long long n, int chunk, int* __restrict__ perm) {
  extern __shared__ double smem[];
  __shared__ int wtot[4];
  const InstDev& d = insts[slot];
  const long long c0 = (long long)blockIdx.x * chunk;
  const long long rem = n - c0;
  const int m = (int)(rem < (long long)chunk ? rem : (long long)chunk);
  T* stagebuf = reinterpret_cast<T*>(smem);                                   // chunk T
  unsigned short* kA = reinterpret_cast<unsigned short*>(stagebuf + chunk);   // 4 x chunk
  unsigned short* kB = kA + chunk;
  unsigned short* iA = kB + chunk;
  unsigned short* iB = iA + chunk;
  int* cnt = reinterpret_cast<int*>(iB + chunk);                              // 32 x 256
  const int tid = threadIdx.x;
  const VPG T* Qp = gp<T>(d.Q);
  for (int k = tid; k < m; k += kBlock) {
    kA[k] = (unsigned short)cell_of((double)Qp[c0 + k] * d.inv_h, d.ng);
    iA[k] = (unsigned short)k;
  }
  __syncthreads();
  const int seg = (m + kBlock - 1) / kBlock;
  const int lo = min(m, tid * seg), hi = min(m, lo + seg);
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = 5 * pass;
    const unsigned short* sk = pass ? kB : kA;
    const unsigned short* si = pass ? iB : iA;
    unsigned short* dk = pass ? kA : kB;
    unsigned short* di = pass ? iA : iB;
    for (int bkt = 0; bkt < 32; ++bkt) cnt[bkt * kBlock + tid] = 0;
    for (int k = lo; k < hi; ++k) cnt[((sk[k] >> shift) & 31) * kBlock + tid] += 1;
    __syncthreads();
    int running = 0;
    for (int bkt = 0; bkt < 32; ++bkt) {
      const int val = cnt[bkt * kBlock + tid];
      int incl = val;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if ((tid & 63) >= off) incl += y;
      }
      if ((tid & 63) == 63) wtot[tid >> 6] = incl;
      __syncthreads();
      int before = 0;
      for (int w = 0; w < (tid >> 6); ++w) before += wtot[w];
      const int total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
      cnt[bkt * kBlock + tid] = running + before + incl - val;
      running += total;
      __syncthreads();
    }
    for (int k = lo; k < hi; ++k) {
      const int bkt = (sk[k] >> shift) & 31;
      const int pos = cnt[bkt * kBlock + tid]++;
      dk[pos] = sk[k];
      di[pos] = si[k];
    }
    __syncthreads();
  }
  if (perm)
    for (int k = tid; k < m; k += kBlock) perm[c0 + k] = (int)(c0 + iA[k]);
  permute_array<T>(gp<T>(d.Q), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.P), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.qs), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.ps), c0, m, iA, stagebuf);
  permute_array<T>(gp<T>(d.psi), c0, m, iA, stagebuf);
}

// ------------------------------------------------------------------ host launchers
static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout workspace_layout(int ng, int order, int hist_cap, long long n) {
  WsLayout w{};
  size_t o = 0;
  const size_t nacc = (size_t)(order == 2 ? 2 : 1) * ng;
  w.acc = o;     o = align256(o + (size_t)kRing * VP_MAX_ACC_COPIES * nacc * sizeof(double));
  w.E = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.g = o;       o = align256(o + (size_t)ng * sizeof(double));
  w.Ef = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.gf = o;      o = align256(o + (size_t)ng * sizeof(float));
  w.Phi = o;     o = align256(o + nacc * sizeof(double));
  w.bt = o;      o = align256(o + nacc * sizeof(double));
  w.tw = o;      o = align256(o + (size_t)ng * sizeof(double));
  w.inv_lam = o; o = align256(o + (size_t)ng * sizeof(double));
  w.cw = o;      o = align256(o + (size_t)kConsTapsMax * sizeof(double));
  w.scal = o;    o = align256(o + sizeof(InstScal));
  w.hist = o;    o = align256(o + (size_t)hist_cap * kHistFields * sizeof(double));
  w.kin = o;     o = align256(o + (size_t)kRing * kin_capacity(n) * kKinFields * sizeof(double));
  w.total = o;
  return w;
}

int kin_capacity(long long n) { return (int)((n + kMinTile - 1) / kMinTile); }

size_t particle_lds_bytes(int /*mode*/, int max_ng) {
  return lds_doubles_per_node() * (size_t)max_ng * sizeof(double);
}

#define VP_DISPATCH(mode, tpb, KERNEL, ...)                                                  \
  do {                                                                                       \
    if ((mode) == kFP32TwoSum) {                                                             \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 1024>), __VA_ARGS__);       \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 512>), __VA_ARGS__);    \
      else hipLaunchKernelGGL((KERNEL<kFP32TwoSum, 256>), __VA_ARGS__);                      \
    } else if ((mode) == kFP64) {                                                            \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP64, 1024>), __VA_ARGS__);             \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP64, 512>), __VA_ARGS__);          \
      else hipLaunchKernelGGL((KERNEL<kFP64, 256>), __VA_ARGS__);                            \
    } else if ((mode) == kFP32Comp) {                                                        \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32Comp, 1024>), __VA_ARGS__);         \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32Comp, 512>), __VA_ARGS__);      \
      else hipLaunchKernelGGL((KERNEL<kFP32Comp, 256>), __VA_ARGS__);                        \
    } else {                                                                                 \
      if ((tpb) == 1024) hipLaunchKernelGGL((KERNEL<kFP32, 1024>), __VA_ARGS__);             \
      else if ((tpb) == 512) hipLaunchKernelGGL((KERNEL<kFP32, 512>), __VA_ARGS__);          \
      else hipLaunchKernelGGL((KERNEL<kFP32, 256>), __VA_ARGS__);                            \
    }                                                                                        \
  } while (0)

hipError_t launch_fused(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, bool lds_fft, int phase, bool dipoles,
                        bool general, bool p2, bool moments, hipStream_t s) {
  switch (mode) {
    case kFP64:
      return launch_fused_mode<kFP64>(tpb, d_inst, d_tiles, tile0, ntiles, ppt, max_ng, lds_fft,
                                      phase, dipoles, general, p2, moments, s);
    case kFP32Comp:
      return launch_fused_mode<kFP32Comp>(tpb, d_inst, d_tiles, tile0, ntiles, ppt, max_ng,
                                          lds_fft, phase, dipoles, general, p2, moments, s);
    case kFP32:
      return launch_fused_mode<kFP32>(tpb, d_inst, d_tiles, tile0, ntiles, ppt, max_ng, lds_fft,
                                      phase, dipoles, general, p2, moments, s);
    default:
      return launch_fused_mode<kFP32TwoSum>(tpb, d_inst, d_tiles, tile0, ntiles, ppt, max_ng,
                                            lds_fft, phase, dipoles, general, p2, moments, s);
  }
}


hipError_t launch_deposit(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_deposit, dim3(ntiles), dim3(tpb), particle_lds_bytes(mode, max_ng), s,
              d_inst, d_tiles, tile0, ppt, phase);
  return hipGetLastError();
}

hipError_t launch_gather_push(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles,
                              int tile0, int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, kick, drift, 0,
              0);
  return hipGetLastError();
}

hipError_t launch_settle(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_gather_push, dim3(ntiles), dim3(tpb),
              (size_t)2 * max_ng * sizeof(double), s, d_inst, d_tiles, tile0, ppt, 0.0, 0.0, 1,
              phase);
  return hipGetLastError();
}

hipError_t launch_diag(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, int phase, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  VP_DISPATCH(mode, tpb, k_diag, dim3(ntiles), dim3(tpb), (size_t)2 * max_ng * sizeof(double), s,
              d_inst, d_tiles, tile0, ppt, phase);
  return hipGetLastError();
}

hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, bool lds_fft, int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  if (mode == kFP64 || mode == kFP32TwoSum)
    hipLaunchKernelGGL(k_solve<kFP64>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst, d_slots,
                       phase);
  else if (mode == kFP32Comp)
    hipLaunchKernelGGL(k_solve<kFP32Comp>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst,
                       d_slots, phase);
  else
    hipLaunchKernelGGL(k_solve<kFP32>, dim3(nslots), dim3(kSolveThreads), lds, s, d_inst, d_slots,
                       phase);
  return hipGetLastError();
}

hipError_t launch_ring(int mode, const InstDev* d_inst, const int* d_slots, int nslots, int op,
                       int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  if (mode == kFP32)
    hipLaunchKernelGGL(k_ring<float>, dim3(nslots), dim3(256), 0, s, d_inst, d_slots, op, phase);
  else
    hipLaunchKernelGGL(k_ring<double>, dim3(nslots), dim3(256), 0, s, d_inst, d_slots, op, phase);
  return hipGetLastError();
}

hipError_t launch_slot_scalars(const InstDev* d_inst, const int* d_slots, int nslots, int op,
                               int phase, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_scalars, dim3((nslots + 63) / 64), dim3(64), 0, s, d_inst, d_slots,
                     nslots, op, phase);
  return hipGetLastError();
}

hipError_t launch_slot_status(const InstDev* d_inst, const int* d_slots, int nslots,
                              long long* out, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_status, dim3((nslots + 63) / 64), dim3(64), 0, s, d_inst, d_slots,
                     nslots, out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  // bytes: a multiple of 4 (whole float or double elements)
  const size_t n8 = bytes / 8;
  const bool tail4 = (bytes % 8) >= 4;
  if (n8 == 0 && !tail4) return hipSuccess;
  size_t blocks = (n8 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<unsigned long long*>(p), n8, tail4);
  return hipGetLastError();
}

hipError_t launch_cell_index(const InstDev* d_inst, int slot, int mode, int* cells, long long n,
                             hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (mode == kFP64)
    hipLaunchKernelGGL(k_cell_index<double>, dim3((unsigned)blocks), dim3(256), 0, s, d_inst, slot,
                       cells, n);
  else
    hipLaunchKernelGGL(k_cell_index<float>, dim3((unsigned)blocks), dim3(256), 0, s, d_inst, slot,
                       cells, n);
  return hipGetLastError();
}

hipError_t launch_sort(int mode, const InstDev* d_inst, int slot, long long n, int chunk,
                       int* perm, hipStream_t s) {
  const long long blocks = (n + chunk - 1) / chunk;
  if (blocks <= 0) return hipSuccess;
  const size_t tsz = (mode == kFP64) ? sizeof(double) : sizeof(float);
  const size_t lds = (size_t)chunk * tsz + (size_t)4 * chunk * sizeof(unsigned short) +
                     (size_t)32 * kBlock * sizeof(int);
  if (mode == kFP64)
    hipLaunchKernelGGL(k_sort<double>, dim3((unsigned)blocks), dim3(kBlock), lds, s, d_inst, slot,
                       n, chunk, perm);
  else
    hipLaunchKernelGGL(k_sort<float>, dim3((unsigned)blocks), dim3(kBlock), lds, s, d_inst, slot,
                       n, chunk, perm);
  return hipGetLastError();
}

}  // namespace vpk
