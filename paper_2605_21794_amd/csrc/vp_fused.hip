// The fused step kernel (k_fused) of the decorated-particle cycle, with its launch for one
// precision mode.  This unit is compiled once per mode (VP_FUSED_MODE = 0..3, the vpk::Mode
// values), so the modes' kernel instances build side by side.
#include "vp_device.h"

#ifndef VP_FUSED_MODE
#error "compile with -DVP_FUSED_MODE=<mode>"
#endif

namespace vpk {

// DIP = false: every tile of the launch belongs to a monopole-only instance; p* and q* are
// neither read nor written (20 bytes of particle traffic per update instead of 36).
// GEN = false: no instance of the launch has general options (d.general), so the field on a
// particle is read straight from the mesh arrays.  P2 = true: the launch's instances have P2
// elements (separate instances keep the others' registers as they were).
template <int MODE, int TPB, bool DIP, bool GEN, bool P2, bool KM = false>
__global__ __launch_bounds__(TPB) void k_fused(const InstDev* __restrict__ insts,
                                               const Tile* __restrict__ tiles, int tile0,
                                               int ppt, int phase) {
  extern __shared__ double smem[];
  __shared__ double red[4 * (TPB / 64)];
  __shared__ double sred[kSolveRed];
  using T = typename StateType<MODE>::T;
  constexpr int kGroup = group_of<MODE, TPB>();
  const Tile tl = tiles[tile0 + blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  const int r0 = phase, r1 = ring_next(phase), r2 = ring_prev(phase);
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  const int nacc = P2 ? d.nacc : ng;  // load-vector nodes (2 ng for P2)
  double* fE = smem;
  double* fG = smem + ng;
  double* sacc = smem + 2 * ng;
  double* bt = sacc + nacc;
  double* fft = bt + ng;
  VPG InstScal* sc = gp(d.scal);
  // An instance whose diagnostics went NaN / Inf is frozen: its state is no longer a
  // solution, and its particles would all land in element 0.  (Uniform per workgroup.)  The
  // flag is tested once the first loads are out, so its latency overlaps theirs.
  const int frozen = sc->nonfinite;
  const bool first = tl.local == 0;  // the instance's bookkeeping tile (uniform per workgroup)

  // one group of particles per thread: thread t takes tile.begin + k * TPB + t, k0 <= k < k0 + kGroup
  // KM: a launch of k = 3 instances (particles with second moments; P2, general options,
  // never kFP32), whose moments travel with the group
  static_assert(!KM || (GEN && P2 && DIP && MODE != kFP32), "second moments need P2 and GEN");
  constexpr bool kM = KM;
  constexpr int kMG = kM ? kGroup : 1;
  struct Group {
    T q[kGroup], p[kGroup], a[kGroup], b[kGroup], w[kGroup];
    T m[3][kMG];
    long long idx[kGroup];
    bool v[kGroup];
  };
  constexpr bool k3 = kM;
  VPG T* __restrict__ Mqp_ = gp<T>(d.Mqq);
  VPG T* __restrict__ Mqpp = gp<T>(d.Mqp);
  VPG T* __restrict__ Mppp = gp<T>(d.Mpp);
  auto load_group = [&](int k0, Group& g) {
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int loc = (k0 + u) * TPB + (int)threadIdx.x;
      g.v[u] = (k0 + u < ppt) && (loc < tl.count);
      g.idx[u] = tl.begin + loc;
      // every lane loads (a lane past the end of the tile reads the tile's last particle, so
      // no load is under a branch); such a lane then holds an all-zero particle (run_group)
      const long long li = tl.begin + (g.v[u] ? loc : tl.count - 1);
      const T z = T(0);
      const T lq = ntld(Qp + li), lp = ntld(Pp + li), lw = ntld(psip + li);
      g.q[u] = g.v[u] ? lq : z;
      g.p[u] = g.v[u] ? lp : z;
      g.w[u] = g.v[u] ? lw : z;
      g.a[u] = g.b[u] = z;
      if constexpr (DIP) {
        const T la = ntld(qsp + li), lb = ntld(psp + li);
        g.a[u] = g.v[u] ? la : z;
        g.b[u] = g.v[u] ? lb : z;
      }
      if constexpr (kM) {
        g.m[0][u] = g.m[1][u] = g.m[2][u] = T(0);
        if (k3 && g.v[u]) {
          g.m[0][u] = ntld(Mqp_ + g.idx[u]); g.m[1][u] = ntld(Mqpp + g.idx[u]);
          g.m[2][u] = ntld(Mppp + g.idx[u]);
        }
      }
    }
  };

  // The solve's loads go out first and the first group's particle loads right behind them:
  // both latencies overlap, and the solve can start once its own loads are back (the loads
  // return in order) while the particle loads are still in flight.
  SolveIn sin_;
  solve_load<MODE, false, GEN, P2>(d, r0, first, sin_);
  Group g;
  load_group(0, g);
  if (frozen) return;
  for (int j = threadIdx.x; j < nacc; j += TPB) sacc[j] = 0.0;
  const int pend = sc->pend[r0];
  // the first tile records the previous step (if it was a fused step of this instance):
  // its inputs are read now and written after the solve
  long long step = 0;
  double rec[3] = {0.0, 0.0, 0.0};
  if (first) {
    step = sc->step;
    rec[0] = sc->W[r2];
    rec[1] = sc->e1r[r2];
    rec[2] = sc->e1i[r2];
  }
  double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
  {
    double sum[7];
    solve_compute<TPB, GEN, P2>(d, sin_, first, bt, fE, fG, sred, fft, nullptr, sum);
    if (first) {
      const int copies = d.acc_copies;
      for (int c = 0; c < copies; ++c)
        for (int j = threadIdx.x; j < nacc; j += TPB) {
          if constexpr (MODE == kFP32)
            gp<float>(d.acc)[acc_off(d, r2, c) + j] = 0.0f;
          else
            gp(d.acc)[acc_off(d, r2, c) + j] = 0.0;
        }
      if (threadIdx.x == 0) {
        if (pend && step >= 1)
          write_record(d, step - 1, sum[3], sum[4], sum[5], sum[6], rec[0], rec[1], rec[2]);
        sc->W[r0] = sum[0];
        sc->e1r[r0] = sum[1];
        sc->e1i[r0] = sum[2];
        if (!isfinite(sum[0])) sc->nonfinite = 1;
        sc->pend[r1] = 1;
        sc->step = step + 1;
      }
    }
  }

  // Every lane pushes all its particles without a branch: an all-zero particle (a lane past
  // the end of the tile) deposits +0 and adds 0 to the kinetic sums, so the particles'
  // dependency chains interleave; only the stores test the lane.
  auto run_group = [&](Group& g) {
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      T Q = g.q[u], P = g.p[u], qs = g.a[u], ps = g.b[u];
      if constexpr (kM) {
        T Mv[3] = {g.m[0][u], g.m[1][u], g.m[2][u]};
        push_particle<MODE, T, DIP, GEN, P2>(d, fE, fG, sacc, pend, Q, P, qs, ps, g.w[u], Ks,
                                             Ms, Cs, Us, k3, Mv);
        g.m[0][u] = Mv[0]; g.m[1][u] = Mv[1]; g.m[2][u] = Mv[2];
      } else {
        push_particle<MODE, T, DIP, GEN, P2>(d, fE, fG, sacc, pend, Q, P, qs, ps, g.w[u], Ks,
                                             Ms, Cs, Us);
      }
      g.q[u] = Q; g.p[u] = P; g.a[u] = qs; g.b[u] = ps;
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if (!g.v[u]) continue;
      ntst(Qp + g.idx[u], g.q[u]); ntst(Pp + g.idx[u], g.p[u]);
      if constexpr (DIP) { ntst(qsp + g.idx[u], g.a[u]); ntst(psp + g.idx[u], g.b[u]); }
      if constexpr (kM)
        if (k3) {
          ntst(Mqp_ + g.idx[u], g.m[0][u]); ntst(Mqpp + g.idx[u], g.m[1][u]);
          ntst(Mppp + g.idx[u], g.m[2][u]);
        }
    }
  };

  run_group(g);
  for (int k0 = kGroup; k0 < ppt; k0 += kGroup) {
    load_group(k0, g);
    run_group(g);
  }

  // kinetic sums: wave trees, one barrier, one thread stores the workgroup totals in this
  // tile's slot (the next pass's first tile adds the slots in tile order)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  Ks = wave_sum(Ks);
  Ms = wave_sum(Ms);
  Cs = wave_sum(Cs);
  if constexpr (GEN) Us = wave_sum(Us);
  if (lane == 0) {
    red[4 * wid] = Ks;
    red[4 * wid + 1] = Ms;
    red[4 * wid + 2] = Cs;
    if constexpr (GEN) red[4 * wid + 3] = Us;
  }
  __syncthreads();  // also completes every LDS deposit of the workgroup
  if (threadIdx.x == 0) {
    double kb = 0.0, mb = 0.0, cbs = 0.0, ub = 0.0;
    for (int w = 0; w < TPB / 64; ++w) {
      kb += red[4 * w];
      mb += red[4 * w + 1];
      cbs += red[4 * w + 2];
      if constexpr (GEN) ub += red[4 * w + 3];
    }
    VPG double* slot = gp(d.kin) + ((size_t)r0 * d.kin_cap + tl.local) * kKinFields;
    slot[0] = kb;
    slot[1] = mb;
    slot[2] = cbs;
    if constexpr (GEN) slot[3] = ub;  // else it stays zero (no potential in this instance)
  }
  flush<MODE, TPB>(d, sacc, r1, tl.local % d.acc_copies);
}



template <int MODE>
hipError_t launch_fused_mode(int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, bool lds_fft, int phase, bool dipoles,
                        bool general, bool p2, bool moments, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (moments && (MODE == kFP32 || !dipoles || !general || !p2)) return hipErrorInvalidValue;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
#define VP_FUSED_K(M, TB, D, G, P)                                                           \
  hipLaunchKernelGGL((k_fused<M, TB, D, G, P>), dim3(ntiles), dim3(TB), lds, s, d_inst,      \
                     d_tiles, tile0, ppt, phase)
#define VP_FUSED(M, TB)                                                                      \
  do {                                                                                       \
    if constexpr (M != kFP32) {                                                              \
      if (moments) {                                                                         \
        hipLaunchKernelGGL((k_fused<M, TB, true, true, true, true>), dim3(ntiles), dim3(TB),   \
                           lds, s, d_inst, d_tiles, tile0, ppt, phase);                      \
        break;                                                                               \
      }                                                                                      \
    }                                                                                        \
    if (dipoles) {                                                                           \
      if (p2) {                                                                              \
        if (general) VP_FUSED_K(M, TB, true, true, true);                                    \
        else VP_FUSED_K(M, TB, true, false, true);                                           \
      } else {                                                                               \
        if (general) VP_FUSED_K(M, TB, true, true, false);                                   \
        else VP_FUSED_K(M, TB, true, false, false);                                          \
      }                                                                                      \
    } else {                                                                                 \
      if (p2) {                                                                              \
        if (general) VP_FUSED_K(M, TB, false, true, true);                                   \
        else VP_FUSED_K(M, TB, false, false, true);                                          \
      } else {                                                                               \
        if (general) VP_FUSED_K(M, TB, false, true, false);                                  \
        else VP_FUSED_K(M, TB, false, false, false);                                         \
      }                                                                                      \
    }                                                                                        \
  } while (0)
#define VP_FUSED_TPB(M)                                                                      \
  do {                                                                                       \
    if (tpb == 1024) VP_FUSED(M, 1024);                                                      \
    else if (tpb == 512) VP_FUSED(M, 512);                                                   \
    else VP_FUSED(M, 256);                                                                   \
  } while (0)
  VP_FUSED_TPB(MODE);
#undef VP_FUSED_TPB
#undef VP_FUSED
#undef VP_FUSED_K
  return hipGetLastError();
}

template hipError_t launch_fused_mode<VP_FUSED_MODE>(int tpb, const InstDev* d_inst,
                                                     const Tile* d_tiles, int tile0, int ntiles,
                                                     int ppt, int max_ng, bool lds_fft, int phase,
                                                     bool dipoles, bool general, bool p2,
                                                     bool moments, hipStream_t s);

}  // namespace vpk
