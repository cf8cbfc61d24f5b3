// dt_track.hpp -- the plain stack by checkpoint prediction: a wavefront of
// 64 orbits walks the exposures in epoch order together.
//
// Sec. 3 / Algorithm 1 test every (image, orbit) pair; almost all pairs miss
// the image, and a miss can be shown from a cheap bound instead of a full
// propagation.  Every CK_SPAN days of epochs (wave-uniform) each orbit is
// solved at the current exposure's epoch t minus a light-time estimate tg:
// the heliocentric position r, velocity v and half acceleration
// h = -mu r / (2 |r|^3) at T = t - tg form a checkpoint, and the one-step
// light-time correction D bounds |tau - tg|.  For a later exposure, D_t =
// t' - t days on, the observer-relative position is predicted as
//     p = r + D_t (v + D_t h) - obs',
// and the exact one (at the emission epoch t' - tau') lies within
//     m = J D_t^3 / 6 + vmax (|tau' - tau| + |tau - tg|) + slack,
// where J = 2 mu vmax / q^3 bounds the jerk on the orbit (|d/dt (r / |r|^3)|
// = sqrt(v^2 + 3 (r.v)^2 / r^2) / r^3 <= 2 |v| / r^3, r >= q the perihelion
// distance, |v| <= vmax the perihelion speed), and the change of light time
// obeys |tau' - tau| <= (vmax + vobs) D_t / (c - vmax) with vobs the patch's
// observer speed bound.  The sky-cone test of the exposure, widened by
// (1 + tan theta) m, then either proves the sample cannot land or queues it.
// Queued samples are solved exactly, as the per-sample walk solves them
// (Kepler from the checkpoint state, light time to LT_LINEAR_MAX, projection,
// nearest pixel), by whichever lanes are free, 64 at a time, and each orbit
// adds its gathered values in epoch order, so the sums equal those of the
// per-sample walk.
//
// The prediction pays while most samples miss.  A wavefront whose orbits land
// often (more than 1 / TRACK_SWITCH_DEN of its lane-exposures queued, once
// TRACK_SWITCH_MIN exposures are tested or its queue is full, e.g. distant
// objects the field follows for months) gives its orbits up when the launch
// allows it:
// it appends its first orbit index to the deferral list and writes nothing;
// a second, persistent kernel walks the deferred wavefronts per sample from
// the first exposure (the per-sample walk's own sky-cone test, no queue).
#pragma once
#include "dt_stack.hpp"

namespace dtk {

constexpr double CK_REACH = 0.3;     // rad: largest Kepler start step taken warm from a checkpoint
constexpr float PRED_SLACK = 1e-9f;  // AU: rounding of the checkpoint state and of the prediction
constexpr int TQ_CAP = 128;          // queued samples per wavefront (< 64 held + 64 pushed)
constexpr int TQ_LIST = 8;           // queued samples per lane between flushes
constexpr int CK_ANCHOR = 8;         // checkpoints between full sincos re-anchors of sin E, cos E
constexpr int TRACK_SWITCH_DEN = 5;  // a wavefront defers above 1/5 of its lane-exposures queued
constexpr int TRACK_SWITCH_MIN = 3;  // exposures tested before the fraction is trusted

// More than 1 / TRACK_SWITCH_DEN of the 64 n_tested lane-exposures queued:
// for an integer count, q > 64 n / 5 exactly when q > floor(64 n / 5).  Plain
// 32-bit arithmetic on wave-uniform counts, so scalar instructions only (the
// walk runs with fewer than 2^25 exposures, so 64 n_tested < 2^31).
__device__ __forceinline__ bool over_switch(int queued, int n_tested) {
  return queued > (int)(((unsigned)n_tested << 6) / (unsigned)TRACK_SWITCH_DEN);
}

// One wavefront's state in LDS: the queue, and each lane's prepared orbit and
// checkpoint Kepler state (read by whichever lane solves that orbit's queued
// samples).  Only the owning wavefront touches it; LDS operations of one
// wavefront complete in issue order, and the accesses are volatile so the
// compiler keeps that order.
struct TrackQueue {
  int ent[TQ_CAP];                 // exposure << 6 | owner lane
  float tg[TQ_CAP];                // light-time estimate (days; a Newton start only)
  float rx[TQ_CAP], ry[TQ_CAP];    // gathered {psi, phi}; {0, 0} when not a valid sample
  unsigned char list[TQ_LIST][64]; // queue slots of each lane, in push order
  double orb[9][64];               // e, n, M0, aP, bQ of each lane's orbit
  double kep[4][64];               // E, sin E, cos E, g at the lane's checkpoint (M = E - e sin E)
  float bnd[3][64];                // j6, l1, vmax of TrackBound, rounded up (vmax -1: never pruned; -inf: not live)
};
typedef __attribute__((address_space(3))) TrackQueue LdsTrackQueue;

// Coefficients of m (times D^3 and D), scaled by 1.1 >= 1 + tan(theta) (cones
// wider than tan(theta) = 0.1 are not used).
struct TrackBound {
  double j6, l1, vmax;
};

__device__ __forceinline__ void track_bound(double a, double e, const Orbit& o, double vobs, TrackBound& b) {
  const double vmax = o.n * a * sqrt((1.0 + e) / (1.0 - e));
  const double iq = 1.0 / (a * (1.0 - e));
  const double acc = MU_SUN * iq * iq;
  b.j6 = 1.1 * (2.0 * MU_SUN * vmax * iq * iq * iq) / 6.0;
  // the light-time term, plus acc x LT_LINEAR_MAX of margin (the checkpoint's
  // r and v are both taken at T, so no epoch mismatch needs it)
  b.l1 = 1.1 * (vmax * (vmax + vobs) / (C_AU_DAY - vmax) + acc * LT_LINEAR_MAX);
  b.vmax = vmax;
}

// The walk of one wavefront.  All 64 lanes call it together; lanes with
// live = false (no orbit, or one outside the domain) carry any valid
// prepared orbit and queue nothing.  P receives each live lane's sums.
//
// Each exposure first runs the service step (wave-uniform): the queued
// samples, 64 at a time, when a checkpoint is due, the queue is half full or
// a lane's list is full, or after the last exposure; then the checkpoint
// solve of every lane when due.  Both are one loop over jobs so the exact
// solve exists once in the code.  Then the cone test of the prediction
// queues the samples that may land.  After a cone test a wavefront of a
// launch that allows it may give its orbits up (*deferred = true; P is then
// meaningless), see the file comment.
//
// REC (debug kernels only): every sample the walk solves exactly is written
// to row rowbase + lane of dbg (the owner's row for queued samples).  DEFER
// false compiles the deferral out (launches that never defer).  TCV keeps the
// checkpoint epoch in a vector register, so that D = t - tc is one
// instruction per exposure rather than a copy and a subtraction (~1 % on the
// stacks that fit it without spilling; the cell and id-list kernels do not).
template <bool REC = false, bool DEFER = true, bool TCV = false>
__device__ __forceinline__ void track_walk(const StackArgs& A, const Orbit& o, const TrackBound& bd, bool live,
                                           TrackQueue& Qm, StackPart& P, bool& deferred,
                                           const DebugArgs* dbg = nullptr, int64_t rowbase = 0) {
  // LDS address space explicitly: volatile accesses through a generic pointer
  // would be kept generic (flat) by the compiler
  volatile LdsTrackQueue& Q = *(volatile LdsTrackQueue*)(&Qm);
  const int lane = (int)__lane_id();
  GExpMeta* __restrict__ meta = global_meta(A.meta);
  P.ps.init();
  P.ph.init();
  P.nv = 0;
  if (A.n_exp <= 0) return;
  Q.orb[0][lane] = o.e;
  Q.orb[1][lane] = o.n;
  Q.orb[2][lane] = o.m0;
  Q.orb[3][lane] = o.aP0;
  Q.orb[4][lane] = o.aP1;
  Q.orb[5][lane] = o.aP2;
  Q.orb[6][lane] = o.bQ0;
  Q.orb[7][lane] = o.bQ1;
  Q.orb[8][lane] = o.bQ2;
  // An orbit whose bound coefficients do not fit FP32 comfortably (perihelion
  // distance ~1e-10 AU, absurd observer speeds) is never pruned: its slack
  // stays 1e300 and the stored coefficients are 0, so no step of zero
  // multiplies an infinity.
  const bool bounded = bd.j6 < 1e30 && bd.l1 < 1e30 && bd.vmax < 1e30;
  Q.bnd[0][lane] = bounded ? __double2float_ru(bd.j6) : 0.f;
  Q.bnd[1][lane] = bounded ? __double2float_ru(bd.l1) : 0.f;
  Q.bnd[2][lane] = !live ? -__builtin_inff() : bounded ? __double2float_ru(bd.vmax) : -1.f;  // read at checkpoints
  double j6 = 0.0, l1 = 0.0;  // reloaded after every service step
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, v0 = 0.0, v1 = 0.0, v2 = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
  float s0 = 0.f;    // slack (AU, rounded up); +inf: not pruned at this checkpoint; -inf: lane not live
  double tc = 0.0;   // checkpoint epoch
  int ck_at = 0;     // exposure of the next checkpoint (the last one's ck_next: the first more than CK_SPAN on)
  int n_ck = 0;      // checkpoints so far
  int count = 0;     // queued samples (wave-uniform)
  int len = 0;       // this lane's queued samples
  int queued = 0;    // samples queued so far (wave-uniform)
  int svc_at = 0;    // step of the next service: the next checkpoint, the final step, or the one after the queue filled
  int ex = 0;
  int n_tested = 0;  // exposures tested by prediction (wave-uniform)
  bool tail = false; // give the orbits up for the per-sample walk
  const bool may_defer = DEFER && A.defer_list != nullptr;

  for (;; ++ex) {
    // the step after the last exposure only serves the queue; the record
    // after the last one repeats it, so it is read like any other
    GExpMeta& x = meta[ex];
    // the cone of this exposure read now, with the epoch and observer, so
    // both loads are in flight together
    double ux = x.ux, uy = x.uy, uz = x.uz, ctan = x.cone_tan, clim = x.cone_lim;
    double D = x.t - tc;
    double p0 = fma(fma(h0, D, v0), D, r0) - x.ox;
    double p1 = fma(fma(h1, D, v1), D, r1) - x.oy;
    double p2 = fma(fma(h2, D, v2), D, r2) - x.oz;
    // one integer compare decides whether this step serves (svc_at <= n_exp,
    // so the final step always does)
    if (ex >= svc_at) {
      const bool last = ex == A.n_exp;
      // D > CK_SPAN, precomputed per exposure (ck_next: the same subtraction,
      // non-decreasing along the epochs); "none" is n_exp + 1, so the final
      // step never takes a checkpoint
      const bool ck = ex >= ck_at;
      const bool fl = count > 0;
      // a wavefront due to serve its queue whose queued fraction is already
      // above 1 / TRACK_SWITCH_DEN defers now rather than solve samples the
      // per-sample walk repeats
      tail = may_defer && fl && !last && over_switch(queued + count, n_tested);
      if (tail) break;
      const int nb = fl ? (count + 63) >> 6 : 0;
      float tg_ck = 0.f;  // a Newton start only
      if (ck && ex > 0) {
        const double d2 = fma(p0, p0, fma(p1, p1, p2 * p2));
        tg_ck = (float)(d2 * __builtin_amdgcn_rsq(d2) * IC);
      }
#pragma unroll 1
      for (int jb = 0; jb < nb + (ck ? 1 : 0); ++jb) {
        const bool ckj = jb == nb;  // the checkpoint job comes last
        const int i = jb * 64 + lane;
        const bool has = ckj || i < count;
        const int ent = ckj ? ((ex << 6) | lane) : (has ? Q.ent[i] : lane);
        const int L = ent & 63;
        if (has) {
          Orbit oo;
          KepState kk;
          oo.e = Q.orb[0][L];
          oo.n = Q.orb[1][L];
          oo.m0 = Q.orb[2][L];
          oo.aP0 = Q.orb[3][L];
          oo.aP1 = Q.orb[4][L];
          oo.aP2 = Q.orb[5][L];
          oo.bQ0 = Q.orb[6][L];
          oo.bQ1 = Q.orb[7][L];
          oo.bQ2 = Q.orb[8][L];
          kk.E = Q.kep[0][L];
          kk.sE = Q.kep[1][L];
          kk.cE = Q.kep[2][L];
          kk.g = Q.kep[3][L];
          kk.M = fma(-oo.e, kk.sE, kk.E);  // the solved equation, to the Newton tolerance
          GExpMeta& xm = meta[ent >> 6];
          const double dt = xm.t - A.epoch;
          const double b0 = -xm.ox, b1 = -xm.oy, b2 = -xm.oz;
          double tg = (double)(ckj ? tg_ck : Q.tg[i]);
          // exact solve: Kepler (cold at the first exposure, else warm from the
          // checkpoint state, re-anchored every CK_ANCHOR checkpoints), light time
          double M = fma(oo.n, dt - tg, oo.m0);
          kepler_general(M, oo.e, kk, ckj && n_ck % CK_ANCHOR == CK_ANCHOR - 1, ckj && ex == 0, CK_REACH);
          LtSolve s;
          lt_state(oo, kk, b0, b1, b2, tg, s);
          // a checkpoint after the first needs no converged light time (see below)
          if ((!ckj || ex == 0) && !(fabs(s.D) <= LT_LINEAR_MAX)) {
#pragma unroll 1
            for (int pass = 1; pass <= 3; ++pass) {
              tg += s.D;
              M = fma(oo.n, dt - tg, oo.m0);
              kepler_general(M, oo.e, kk, false, false);
              lt_state(oo, kk, b0, b1, b2, tg, s);
              if (fabs(s.D) <= LT_LINEAR_MAX) break;
            }
          }
          if (ckj) {
            // New checkpoint: the state at T = t - tg (the prediction state is
            // rebuilt from it below).  The exact emission epoch of this
            // exposure is T - D up to the one-step error, so predictions taken
            // at t_j - tg are off by at most vmax (|tau_j - tau_c| + |D|): the
            // second part goes into the slack.
            Q.kep[0][lane] = kk.E;
            Q.kep[1][lane] = kk.sE;
            Q.kep[2][lane] = kk.cE;
            Q.kep[3][lane] = kk.g;
            // in FP32 (no FP64 constants held across the walk): each of the
            // three roundings is below 1e-7 relative, and the factor
            // 1.1 * (1 + 1e-6) keeps s0 above 1.1 (PRED_SLACK + vmax dtau)
            const float dtau = fmaf(1.01f, fabsf((float)s.D), 1e-9f);
            // a lane that is not live gets -inf: its cone test never passes
            const float vmax = Q.bnd[2][lane];
            s0 = vmax >= 0.f && dtau < 1.f ? 1.1000011f * fmaf(vmax, dtau, PRED_SLACK)
                                           : vmax < -1.f ? -__builtin_inff() : __builtin_inff();
          } else {
            SampleOut so;
            project((const ExpMeta&)xm, s, so);
            float2 v = make_float2(0.f, 0.f);
            if (so.inside) v = global_load(A.planes, xm.plane_off + (int64_t)so.iy * xm.W + so.ix);
            const bool ok = v.y > 0.f;
            Q.rx[i] = ok ? v.x : 0.f;
            Q.ry[i] = ok ? v.y : 0.f;
            if (REC) {
              so.tau = tg + s.D;
              rec_sample(*dbg, A.n_exp, rowbase + L, (const ExpMeta&)xm, so, v);
            }
          }
        }
      }
      if (nb > 0) {
        // each orbit adds its samples in push (= epoch) order
#pragma unroll 1
        for (int q = 0; q < len; ++q) {
          const int i = Q.list[q][lane];
          const float vx = Q.rx[i], vy = Q.ry[i];
          if (vy > 0.f) {
            P.ps.add(vx);
            P.ph.add(vy);
            P.nv++;
          }
        }
        queued += count;
        count = 0;
        len = 0;
      }
      // prediction state from the checkpoint kept in LDS (recomputed after every
      // service step, so it holds no registers while the solves run): the
      // heliocentric position r(E) and velocity v(E) at T and the half
      // acceleration -mu r / (2 |r|^3)
      {
        const double e = Q.orb[0][lane], n = Q.orb[1][lane];
        const double aP0 = Q.orb[3][lane], aP1 = Q.orb[4][lane], aP2 = Q.orb[5][lane];
        const double bQ0 = Q.orb[6][lane], bQ1 = Q.orb[7][lane], bQ2 = Q.orb[8][lane];
        const double sE = Q.kep[1][lane], cE = Q.kep[2][lane], g = Q.kep[3][lane];
        const double cme = cE - e, ng = n * g;
        const double vs = -ng * sE, vc = ng * cE;
        v0 = fma(vc, bQ0, vs * aP0);
        v1 = fma(vc, bQ1, vs * aP1);
        v2 = fma(vc, bQ2, vs * aP2);
        r0 = fma(cme, aP0, sE * bQ0);
        r1 = fma(cme, aP1, sE * bQ1);
        r2 = fma(cme, aP2, sE * bQ2);
        double rr, irr;
        sqrt_rsq(fma(r0, r0, fma(r1, r1, r2 * r2)), rr, irr);
        const double hk = -0.5 * MU_SUN * irr * irr * irr;
        h0 = hk * r0;
        h1 = hk * r1;
        h2 = hk * r2;
        j6 = (double)Q.bnd[0][lane];
        l1 = (double)Q.bnd[1][lane];
      }
      // this exposure's record again, by an index the compiler does not
      // match with the first one (ex >> 30 is 0), so the first values need
      // not be kept in registers across the solves
      GExpMeta& y = meta[ex + (ex >> 30)];
      if (ck) {
        tc = y.t;
        if (TCV) asm volatile("" : "+v"(tc));
        ck_at = y.ck_next;
        n_ck++;
        D = 0.0;
      }
      p0 = fma(fma(h0, D, v0), D, r0) - y.ox;
      p1 = fma(fma(h1, D, v1), D, r1) - y.oy;
      p2 = fma(fma(h2, D, v2), D, r2) - y.oz;
      ux = y.ux;  // the cone again too: nothing of the first read stays live across the solves
      uy = y.uy;
      uz = y.uz;
      ctan = y.cone_tan;
      clim = y.cone_lim;
      svc_at = ck_at < A.n_exp ? ck_at : A.n_exp;
      if (last) break;
    }
    n_tested++;
    // cone test of the prediction (bitwise logic, no branches)
    const double sc = fma(ux, p0, fma(uy, p1, uz * p2));
    const double d2 = fma(p0, p0, fma(p1, p1, p2 * p2));
    const double m = fma(fma(j6, D * D, l1), D, (double)s0);
    const double R = fma(ctan, sc, m);
    const bool in_front = R >= 0.0, in_cone = fma(-R, R, fma(-sc, sc, d2)) <= clim;
    const bool may = in_front & in_cone;
    // the mask from one ballot per compare (each is the compare's own lane
    // mask; a ballot of the combined flag would rebuild it from a vector)
    const uint64_t mask = __builtin_amdgcn_ballot_w64(in_front) & __builtin_amdgcn_ballot_w64(in_cone);
    if (mask) {
      if (may) {
        const int slot = count + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        Q.ent[slot] = (ex << 6) | lane;
        Q.tg[slot] = (float)(d2 * __builtin_amdgcn_rsq(d2) * IC);
        Q.list[len][lane] = (unsigned char)slot;
        len++;
      }
      count += __builtin_popcountll(mask);
      // a full queue (or a lane's list) is served at the next step
      const bool full = count >= 64 || __builtin_amdgcn_ballot_w64(len >= TQ_LIST) != 0;
      if (full) svc_at = ex + 1;
      // most samples may land: leave these orbits to the per-sample walk
      // (nothing queued is served).  A queue that fills before
      // TRACK_SWITCH_MIN exposures decides at once, rather than serving
      // solves the per-sample walk would repeat.
      tail = may_defer && (n_tested >= TRACK_SWITCH_MIN || full) && over_switch(queued + count, n_tested);
      if (tail) break;
    }
  }
  deferred = tail;
  const unsigned long long nl = (unsigned long long)__builtin_popcountll(__builtin_amdgcn_ballot_w64(live));
  if (A.work && lane == 0) {
    // wave totals (uniform values) into this workgroup's slot
    unsigned long long* w = A.work + WORK_N * (blockIdx.x % WORK_SLOTS);
    atomicAdd(w + WORK_PRED, nl * (unsigned long long)n_tested);
    atomicAdd(w + WORK_QUEUED, (unsigned long long)queued);
    atomicAdd(w + WORK_CKPT, nl * (unsigned long long)n_ck);
    if (tail) atomicAdd(w + WORK_SWITCHED, 1ull);
  }
}

// One lane's orbit through the walk of its wavefront: `el` holds the
// elements when `live` (any values otherwise); the outputs are those of the
// per-sample stack (NaN, NaN, -1 for an orbit that is not live), or nothing
// when the wavefront deferred its orbits (returns true).  All 64 lanes of the
// wavefront call it together; Q is the wavefront's LDS queue.
template <bool REC = false, bool DEFER = true, bool TCV = false>
__device__ __forceinline__ bool track_stack_lane(const StackArgs& A, const double el[6], bool live, TrackQueue& Q,
                                                 float& snr, float& flux, int& nv, const DebugArgs* dbg = nullptr,
                                                 int64_t rowbase = 0) {
  double a = el[0], e = el[1], inc = el[2], node = el[3], peri = el[4], m0 = el[5];
  if (!live) {
    a = 2.5;
    e = inc = node = peri = m0 = 0.0;
  }
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  TrackBound bd;
  track_bound(a, e, ob, A.vobs, bd);
  StackPart P;
  bool deferred = false;
  track_walk<REC, DEFER, TCV>(A, ob, bd, live, Q, P, deferred, dbg, rowbase);
  snr = flux = __builtin_nanf("");
  nv = -1;
  if (deferred) return true;
  if (live) stack_finish(P, snr, flux, nv);
  return false;
}

// First global thread index of the calling wavefront, from wave-uniform parts
// only (scalar registers), so that no 64-bit per-lane index has to stay live
// in vector registers through the walk.
__device__ __forceinline__ int64_t wave_base() {
  return (int64_t)blockIdx.x * blockDim.x + (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x & ~63u);
}

// This lane's global thread index again after the walk, from the wave-uniform
// base and an opaque copy of the lane id, so that the compiler cannot reuse
// (and therefore keep live, or spill) the index computed before the walk.
__device__ __forceinline__ int64_t thread_index_after_walk() {
  int lane = (int)__lane_id();
  asm volatile("" : "+v"(lane));
  return wave_base() + lane;
}

// A deferring wavefront's list entry: its first orbit index (lane 0 writes).
__device__ __forceinline__ void defer_wave(const StackArgs& A, int64_t first) {
  if (__lane_id() == 0) {
    const unsigned int slot = atomicAdd(A.defer_count, 1u);
    A.defer_list[slot] = first;
  }
}

// Per-sample walk of orbit o (its elements el, valid when live) for the
// deferred wavefronts: the walk of stack_walk, with the work counters.
__device__ __forceinline__ void deferred_lane(const StackArgs& A, const double el[6], bool live, float& snr,
                                              float& flux, int& nv) {
  snr = flux = __builtin_nanf("");
  nv = -1;
  StackPart P;
  int n_full = 0;
  if (live) {
    Orbit ob;
    orbit_prep(el[0], el[1], el[2], el[3], el[4], el[5], ob);
    stack_range(A, ob, 0, A.n_exp, P, nullptr, 0, n_full);
    stack_finish(P, snr, flux, nv);
  }
  if (A.work) {
    const unsigned long long nl = (unsigned long long)__builtin_popcountll(__builtin_amdgcn_ballot_w64(live));
    int tot = n_full;  // wavefront sum
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) tot += __shfl_xor(tot, m, 64);
    if (__lane_id() == 0) {
      unsigned long long* w = A.work + WORK_N * (blockIdx.x % WORK_SLOTS);
      atomicAdd(w + WORK_TAIL, nl * (unsigned long long)A.n_exp);
      atomicAdd(w + WORK_TAIL_FULL, (unsigned long long)tot);
    }
  }
}

}  // namespace dtk
