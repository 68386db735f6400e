// The persistent form of the fused step (k_persist): many steps in one cooperative launch,
// the particles of each tile held in registers, with its launch and capacity query.
#include "vp_device.h"

namespace vpk {

// ------------------------------------------------------------------ persistent step
// nsteps fused steps in one cooperative launch (every workgroup resident at once).  The
// particles of each tile stay in registers from the first step to the last.  Between steps
// every workgroup of an instance waits until all of the instance's tiles have flushed the
// previous step, through the two-level arrival tree of InstScal: group counters, a top
// counter, and release flags written by the tile that completes the top counter; one lane
// of each waiting tile polls one flag, with a bounded spin (after d.spin_limit polls the
// instance is flagged, the wait ends and that tile waits no more in this launch, so every
// wave finishes within one such period).  Data other workgroups of the launch wrote (the load
// vector, the per-tile kinetic sums, the cleared ring entry) is read and written at device
// scope.  The ring protocol, the records and the arithmetic are those of k_fused, so nsteps
// persistent steps equal nsteps fused launches.  A launch with a P2 instance takes the P2
// instance of the kernel (which runs its P1 instances too); particles with second moments
// are not taken (the host refuses persistent tuning for them).
//
// What no other tile needs is kept off the path between the barriers: every tile clears its
// own slice of the ring entry the next step deposits into, and the instance's first tile
// writes the record of step n-1 and the field summary of step n after it has counted its
// arrival for step n, while the others are still on their way.  That bookkeeping is done by
// the tile's first wavefront alone, with no workgroup barrier (its last wavefront polls the
// release meanwhile), and reads LDS only: the first tile copies the Fourier weights of E1 to
// LDS once per launch, and issues the loads of the previous pass's per-tile kinetic sums
// together with the solve's loads, parking the per-thread partials in LDS after the solve
// (device-scope loads after the arrival would hold it past the others' release).
// GEN = false: no instance of the launch has general options (fewer registers).

// The first tile's bookkeeping after step n, by its first wavefront alone (no workgroup
// barrier, so the tile's other waves go on to the next step's wait): the field summary of
// the field in LDS (W, E1), into rec and the instance's field-summary ring entry r0; and,
// when write_rec, the record of integer step rec_step with the kinetic sums of the previous
// pass (skin: each solving thread's partial sums, field f of thread t at
// f * kSolveThreads + t, as load_kin forms them from the per-tile slots) and the field
// summary rec of that step, into history slot rec_slot (rec_step mod hist_cap).  Each lane
// takes nodes and partials lane, lane + 64, ... in order, then one wave tree per quantity: a
// fixed order.  The node loop is unrolled by four (the loads of four nodes go out together;
// the additions keep their order) and the seven trees run side by side (wave_sum_n): this
// wave's work delays the tile's next step.  tw: the Fourier weights (d.tw) in LDS.  rec is
// read and updated in every lane (the wave trees leave the totals in all).
template <bool GEN, bool P2>
__device__ void persist_bookkeeping(const InstDev& d, const double* fE, const double* fG,
                                    const double* tw, const double* skin, int r0,
                                    bool write_rec, long long rec_step, int rec_slot,
                                    double (&rec)[3]) {
  const int ng = d.ng, lane = threadIdx.x & 63;
  // v: W's sum, E1 real and imaginary, then the kinetic fields
  double v[3 + kKinFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (write_rec)
#pragma unroll
    for (int k = 0; k < kSolveThreads / 64; ++k)
#pragma unroll
      for (int f = 0; f < kKinFields; ++f) v[3 + f] += skin[f * kSolveThreads + lane + 64 * k];
  const int halfn = ng >> 1;
  for (int base = 0; base < ng; base += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + 64 * u + lane;
      if (e < ng) {
        const int t = e & (halfn - 1);
        const double sg = (e < halfn) ? 1.0 : -1.0;  // cos / sin of theta + pi
        const double c = sg * tw[2 * t], sn = sg * tw[2 * t + 1];
        const double Ee = fE[e];
        v[0] += Ee * Ee;
        v[1] += Ee * c;
        v[2] -= Ee * sn;
      }
    }
  }
  if (P2 && d.order == 2) {
    // the field is linear on a P2 element: W gains (1/2) h (3/16) sum b~_m^2 over the
    // midpoint loads, b~_m = -(2h/3) g_e
    double gm = 0.0;
    for (int e = lane; e < ng; e += 64) gm += fG[e] * fG[e];
    v[0] += 0.1875 * ((4.0 / 9.0) * d.h * d.h) * gm;
  }
  wave_sum_n(v);
  const double W = 0.5 * d.h * v[0];
  const double e1r = v[1] * inv_pow2(d.log2ng), e1i = v[2] * inv_pow2(d.log2ng);
  if (lane == 0) {
    if (write_rec)
      write_record_at(d, rec_slot, rec_step, v[3], v[4], v[5], GEN ? v[6] : 0.0, rec[0],
                      rec[1], rec[2]);
    VPG InstScal* sc = gp(d.scal);
    sc->W[r0] = W;
    sc->e1r[r0] = e1r;
    sc->e1i[r0] = e1i;
    if (!isfinite(W)) sc->nonfinite = 1;
  }
  rec[0] = W;
  rec[1] = e1r;
  rec[2] = e1i;
}

template <int MODE, int TPB, int PPT, bool GEN, bool P2>
__global__ __launch_bounds__(TPB) void k_persist(const InstDev* __restrict__ insts,
                                                 const Tile* __restrict__ tiles, int phase0,
                                                 int nsteps) {
  extern __shared__ double smem[];
  __shared__ double red[4 * (TPB / 64)];
  __shared__ double sred[kSolveRed];
  __shared__ double stw[VP_MAX_NG];                     // first tile: Fourier weights of E1
  __shared__ double skin[kKinFields * kSolveThreads];  // first tile: previous pass's partials
  using T = typename StateType<MODE>::T;
  const Tile tl = tiles[blockIdx.x];
  const InstDev& d = insts[tl.inst];
  const int ng = d.ng;
  VPG T* __restrict__ Qp = gp<T>(d.Q);
  VPG T* __restrict__ Pp = gp<T>(d.P);
  VPG T* __restrict__ qsp = gp<T>(d.qs);
  VPG T* __restrict__ psp = gp<T>(d.ps);
  const VPG T* __restrict__ psip = gp<T>(d.psi);
  const int nacc = P2 ? d.nacc : ng;  // load-vector nodes (2 ng for a P2 instance)
  double* fE = smem;
  double* fG = smem + ng;
  double* sacc = smem + 2 * ng;
  double* bt = sacc + nacc;
  double* fft = bt + ng;
  VPG InstScal* sc = gp(d.scal);
  if (sc->frozen) return;  // fixed for the launch: all tiles of the instance leave together
  const bool first = tl.local == 0;

  // A lane past the end of the tile holds an all-zero particle: its deposit adds +0 and its
  // kinetic sums 0, so every lane runs the push without a branch (only the stores test it).
  T q[PPT], p[PPT], a[PPT], b[PPT], w[PPT];
  bool v[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int loc = u * TPB + (int)threadIdx.x;
    v[u] = loc < tl.count;
    q[u] = p[u] = a[u] = b[u] = w[u] = T(0);
    if (v[u]) {
      const long long i = tl.begin + loc;
      q[u] = ntld(Qp + i); p[u] = ntld(Pp + i); a[u] = ntld(qsp + i);
      b[u] = ntld(psp + i); w[u] = ntld(psip + i);
    }
  }
  // float64 modes without general options carry each particle's element from one step's
  // deposit to the next step's gather
  constexpr bool kCell = !GEN && !P2 && MODE != kFP32;
  int cell[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) cell[u] = kCell ? cell_of((double)q[u] * d.inv_h, ng) : 0;
  const int pend0 = sc->pend[phase0];
  int pend = pend0;
  if (first) {  // visible at the first step's solve barriers
    const VPG double* twg = gp(d.tw);
    for (int j = threadIdx.x; j < ng; j += TPB) stw[j] = twg[j];
  }
  long long step0 = 0;
  double rec[3] = {0.0, 0.0, 0.0};  // field summary of the previous integer step (first tile)
  int rec_slot = 0;                 // (step0 + st - 1) mod hist_cap at step st (first tile)
  if (first) {
    step0 = sc->step;
    rec_slot = (int)(((step0 - 1) % d.hist_cap + d.hist_cap) % d.hist_cap);
    rec[0] = sc->W[ring_prev(phase0)];
    rec[1] = sc->e1r[ring_prev(phase0)];
    rec[2] = sc->e1i[ring_prev(phase0)];
  }
  // this tile's arrival group (local indices congruent mod ngroups), its size, and the
  // release flag it polls
  const int ngroups = min(kArriveGroups, d.ntiles);
  const int my_group = tl.local % ngroups;
  const unsigned group_tiles = (unsigned)((d.ntiles - my_group + ngroups - 1) / ngroups);
  VPG unsigned* const my_counter = sc->arrive + my_group * kArriveStride;
  VPG unsigned* const my_flag = sc->release + (tl.local & (kReleaseFlags - 1)) * kArriveStride;
  // this tile's slice of a ring entry's copies, cleared for the step after next
  const int ncl = d.acc_copies * nacc;
  const int cl_per = (ncl + d.ntiles - 1) / d.ntiles;
  const int cl0 = min(ncl, tl.local * cl_per), cl1 = min(ncl, cl0 + cl_per);

  bool gave_up = false;  // the poller's wait timed out: it waits no more, the launch drains
  const unsigned spin_limit = min(d.spin_limit, kSpinLimit);
  int r0 = phase0;
  for (int st = 0; st < nsteps; ++st) {
    // nothing is hoisted out of the step loop: keeps the step's registers per step
    __asm__ __volatile__("" ::: "memory");
    const int r1 = ring_next(r0), r2 = ring_prev(r0);
    if (st > 0) {  // wait for every tile of the instance to finish the previous step
      // polled by the last wave: the first wave may still be in the first tile's bookkeeping
      if (threadIdx.x == TPB - 64) {
        unsigned it = 0;
        while (!gave_up && __hip_atomic_load(my_flag, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < (unsigned)st) {
          __builtin_amdgcn_s_sleep(1);
          if (++it > spin_limit) {
            __hip_atomic_store(&sc->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gave_up = true;
          }
        }
      }
      __syncthreads();
    }
    SolveIn sin_;
    solve_load<MODE, true, GEN, P2>(d, r0, false, sin_);
    // the first tile's record of step st - 1 sums ring entry r2, which every tile finished
    // before the barrier just passed: its loads go out with the solve's
    const bool write_rec = st > 0 || (pend0 && step0 >= 1);
    double kinv[kKinFields] = {0.0, 0.0, 0.0, 0.0};
    if (first && write_rec && threadIdx.x < kSolveThreads)
      load_kin<true, GEN ? kKinFields : 3>(d, r2, kinv);
    for (int j = threadIdx.x; j < nacc; j += TPB) sacc[j] = 0.0;
    double Ks = 0.0, Ms = 0.0, Cs = 0.0, Us = 0.0;
    {
      double sum[7];
      solve_compute<TPB, GEN, P2>(d, sin_, false, bt, fE, fG, sred, fft, nullptr, sum);
    }
    if (first && threadIdx.x < kSolveThreads)  // read after the arrival's barrier
#pragma unroll
      for (int f = 0; f < kKinFields; ++f) skin[f * kSolveThreads + threadIdx.x] = kinv[f];
    // ring entry r2 was read at the previous step by every tile (they have all passed the
    // barrier since) and is deposited into at the next one (after the next barrier)
    for (int f = cl0 + (int)threadIdx.x; f < cl1; f += TPB) {
      if constexpr (MODE == kFP32)
        gst(gp<float>(d.acc) + acc_off(d, r2, 0) + f, 0.0f);
      else
        gst(gp(d.acc) + acc_off(d, r2, 0) + f, 0.0);
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u)
      push_particle<MODE, T, true, GEN, P2, -1, kCell>(d, fE, fG, sacc, pend, q[u], p[u], a[u],
                                                       b[u], w[u], Ks, Ms, Cs, Us, false,
                                                       nullptr, &cell[u]);
    pend = 1;

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    Ks = wave_sum(Ks);
    Ms = wave_sum(Ms);
    Cs = wave_sum(Cs);
    if constexpr (GEN) Us = wave_sum(Us);
    if (lane == 0) {
      red[4 * wid] = Ks;
      red[4 * wid + 1] = Ms;
      red[4 * wid + 2] = Cs;
      red[4 * wid + 3] = Us;
    }
    __syncthreads();  // also completes every LDS deposit of the workgroup
    if (threadIdx.x == 0) {
      double kb = 0.0, mb = 0.0, cbs = 0.0, ub = 0.0;
      for (int ww = 0; ww < TPB / 64; ++ww) {
        kb += red[4 * ww];
        mb += red[4 * ww + 1];
        cbs += red[4 * ww + 2];
        if constexpr (GEN) ub += red[4 * ww + 3];
      }
      VPG double* slot = gp(d.kin) + ((size_t)r0 * d.kin_cap + tl.local) * kKinFields;
      gst(slot, kb);
      gst(slot + 1, mb);
      gst(slot + 2, cbs);
      gst(slot + 3, ub);
      if (first) sc->pend[r1] = 1;
    }
    flush<MODE, TPB>(d, sacc, r1, tl.local % d.acc_copies);
    if (st + 1 < nsteps) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's flush, slot and clear are performed
      __syncthreads();
      if (threadIdx.x < 64) {  // count the arrival; the last of all releases step st + 1
        const unsigned e = (unsigned)(st + 1);
        unsigned rel = 0;
        if (threadIdx.x == 0) {
          const unsigned old = __hip_atomic_fetch_add(my_counter, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
          if (old + 1u == e * group_tiles) {
            const unsigned g = __hip_atomic_fetch_add(sc->top, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (g + 1u == e * (unsigned)ngroups) rel = 1;
          }
        }
        if (__shfl(rel, 0))  // the flags are written by the whole wavefront
          for (int f = threadIdx.x; f < kReleaseFlags; f += 64)
            __hip_atomic_store(sc->release + f * kArriveStride, e, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (first && threadIdx.x < 64)  // record of step st - 1, field summary of step st
      persist_bookkeeping<GEN, P2>(d, fE, fG, stw, skin, r0, write_rec, step0 + st - 1,
                                   rec_slot, rec);
    if (++rec_slot == d.hist_cap) rec_slot = 0;
    r0 = r1;
  }
  if (first && threadIdx.x == 0) sc->step = step0 + nsteps;
#pragma unroll
  for (int u = 0; u < PPT; ++u)
    if (v[u]) {
      const long long i = tl.begin + u * TPB + (int)threadIdx.x;
      ntst(Qp + i, q[u]); ntst(Pp + i, p[u]); ntst(qsp + i, a[u]); ntst(psp + i, b[u]);
    }
}

#define VP_PERSIST_CASE(M, TB, PP)                                                          \
  if (mode == M && tpb == TB && ppt == PP) {                                                \
    if (p2) {                                                                               \
      if constexpr (M != kFP32)                                                             \
        fn = general ? reinterpret_cast<const void*>(&k_persist<M, TB, PP, true, true>)     \
                     : reinterpret_cast<const void*>(&k_persist<M, TB, PP, false, true>);   \
    } else {                                                                                \
      fn = general ? reinterpret_cast<const void*>(&k_persist<M, TB, PP, true, false>)      \
                   : reinterpret_cast<const void*>(&k_persist<M, TB, PP, false, false>);    \
    }                                                                                       \
  }

// p2: some instance of the launch has P2 elements (float32 naive state has none); such a
// launch takes the P2 instance of the kernel, which runs the P1 instances too.
static const void* persist_fn(int mode, int tpb, int ppt, bool general, bool p2) {
  const void* fn = nullptr;
#define VP_PERSIST_MODE(M)                                                                  \
  VP_PERSIST_CASE(M, 512, 2) VP_PERSIST_CASE(M, 512, 4) VP_PERSIST_CASE(M, 512, 8)          \
  VP_PERSIST_CASE(M, 1024, 2) VP_PERSIST_CASE(M, 1024, 4) VP_PERSIST_CASE(M, 1024, 8)
  VP_PERSIST_MODE(kFP64)
  VP_PERSIST_MODE(kFP32Comp)
  VP_PERSIST_MODE(kFP32)
  VP_PERSIST_MODE(kFP32TwoSum)
#undef VP_PERSIST_MODE
  return fn;
}
#undef VP_PERSIST_CASE

int persist_capacity(int mode, int tpb, int ppt, int max_ng, bool lds_fft, bool general,
                     bool p2) {
  const void* fn = persist_fn(mode, tpb, ppt, general, p2);
  if (!fn) return 0;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  int per_cu = 0, cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tpb, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_persist(int mode, int tpb, int ppt, const InstDev* d_inst, const Tile* d_tiles,
                          int ntiles, int max_ng, bool lds_fft, bool general, bool p2, int phase,
                          int nsteps, hipStream_t s) {
  if (ntiles <= 0 || nsteps <= 0) return hipSuccess;
  const void* fn = persist_fn(mode, tpb, ppt, general, p2);
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = fused_lds_doubles(lds_fft) * (size_t)max_ng * sizeof(double);
  void* args[] = {(void*)&d_inst, (void*)&d_tiles, (void*)&phase, (void*)&nsteps};
  return hipLaunchCooperativeKernel(fn, dim3(ntiles), dim3(tpb), args, (unsigned)lds, s);
}

}  // namespace vpk
