// HIP kernels of the event-driven e-prop library (gfx950, wave64).
//
// Within one iteration the weights are fixed and the gradient of a sample
// is formed from the sample's archived history (paper, Results: the
// event-driven implementation computes the gradient at the first spike
// after each sample from the archived postsynaptic history).  The path is:
//
//   forward, per step t     neuron update (time-driven, eq. lif_update,
//                                      eq. spike-threshold-adaptation, surrogate)
//                           (k_forward_tiled: persistent, tiles of targets with
//                            LDS delay rings; k_neuron_gather: deterministic)
//   after the sample        k_stage_rec_lists (spike-time lists from the bitsets),
//                           k_readout_sums, k_readout_scan (eq. leaky_integrator,
//                                      error signal, loss; backward filter of E)
//                           k_adjoint (per-neuron arrival archive phi)
//                           k_synapse (event-driven synapse gradient)
//                           k_output_reduce
//   end of iteration        k_apply_blk (scatter delivery, rows dense within a tile)
//                           or k_apply_syn,
//                           k_apply_out (GD or Adam)
//
// The synapse gradient.  For a synapse (i -> j, delay D) with arrival
// indicator x^t, e-prop accumulates g = sum_t L_j^t F_kappa(e^t) with
// e^t = psi_j^t (eps_v^t - beta eps_a^t) and the eligibility vector
// eps^t = J^t eps^{t-1} + (x^t, 0) (eq. eligibility-vector-substituted,
// eq. filtered-eligibility-trace).  Exchanging the order of summation (the
// paper's eq. index-flipping applied to the kappa filter, then once more to
// the eligibility recursion) gives, exactly,
//     g = sum over arrivals a of phi_j^a,
//     Lambda_j^t = sum_k B_jk Ebar_k^t,   Ebar_k^t = E_k^t + kappa Ebar_k^{t+1},
//     mu^t = Lambda^t psi^t (1, -beta) + (J^{t+1})^T mu^{t+1},  phi^t = mu^t[0],
// where (J^{t+1})^T = [[alpha, psi^t], [0, rho - psi^t beta]].  phi_j is a
// per-neuron archive built once per sample; each presynaptic arrival then
// costs one archive read, which the synapse adds with Kahan compensation.
// The output gradient likewise is sum over the spikes u of j of Ebar_k^u.
#include "eprop_internal.h"

#include <mutex>

namespace eprop {
namespace {

__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }

// Compensated summation: s + c is the running sum, c holds the low part.
template <typename real>
__device__ inline void kahan_add(real &s, real &c, real x) {
  const real y = x + c;
  const real t = s + y;
  c = y - (t - s);
  s = t;
}

template <typename real>
__device__ inline real surrogate(const DevNet<real> &n, real dv) {
  if (n.surrogate == 1) return n.sg_gamma * exp(-n.sg_beta * fabs(dv));
  return n.sg_gamma * fmax((real)0, (real)1 - n.sg_beta * fabs(dv));
}

// ----------------------------------------------------------------- staging

// Checks the batch's input spikes (range; order with check_order) and sets
// the emission bitsets in_bits[b][s][src].
template <typename real>
__global__ __launch_bounds__(256) void k_stage_in_bits(DevNet<real> n, uint32_t ntr, uint64_t nsp,
                                                       int check_order) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nsp; e += stride) {
    uint32_t lo = 0, hi = ntr;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (n.in_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    const uint32_t b = lo;
    const uint32_t s = n.in_step[e], i = n.in_src[e];
    if (s >= n.T[b] || i >= n.I) {
      atomicOr(&n.ctl[CTL_ERR], ERR_INPUT_RANGE);
      continue;
    }
    if (check_order && e > n.in_ptr[b]) {
      const uint32_t ps = n.in_step[e - 1], pi = n.in_src[e - 1];
      if (!(ps < s || (ps == s && pi < i))) atomicOr(&n.ctl[CTL_ERR], ERR_INPUT_ORDER);
    }
    atomicOr((unsigned long long *)&n.in_bits[((size_t)b * n.Tcap + s) * n.Iw + (i >> 6)],
             1ull << (i & 63u));
  }
}

// in_step_ptr[b][s] = first input spike of trial b with emission step >= s.
template <typename real>
__global__ __launch_bounds__(256) void k_stage_in_step_ptr(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t T = n.T[b];
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s <= T; s += gridDim.x * blockDim.x) {
    uint64_t lo = n.in_ptr[b], hi = n.in_ptr[b + 1];
    while (lo < hi) {
      const uint64_t mid = lo + ((hi - lo) >> 1);
      if (n.in_step[mid] < s) lo = mid + 1; else hi = mid;
    }
    n.in_step_ptr[(size_t)b * (n.Tcap + 1) + s] = lo;
  }
}

// Spike-time lists, ascending, of the 64 sources of one bitset column, by
// one wavefront: lane l reads the column's word of step t0 + l, and 64
// ballots turn the 64 x 64 bit block around, so that each lane then holds
// its source's spikes over those 64 steps.  Steps t_lo .. t_hi - 1; rows
// are `stride` words apart.  Returns the lane's count (writes only if live).
__device__ inline uint32_t column_lists(const uint64_t *col, size_t stride, uint32_t t_lo, uint32_t t_hi,
                                        uint16_t *out, bool live) {
  const uint32_t lane = lane_id();
  uint32_t c = 0;
  for (uint32_t t0 = t_lo; t0 < t_hi; t0 += 64) {
    const uint32_t t = t0 + lane;
    const uint64_t w = t < t_hi ? col[(size_t)t * stride] : 0ull;
    uint64_t mine = 0;
#pragma unroll 8
    for (uint32_t nb = 0; nb < 64; ++nb) {
      const uint64_t m = __ballot((w >> nb) & 1ull);
      mine = lane == nb ? m : mine;
    }
    while (mine) {
      const uint32_t s = (uint32_t)__ffsll((unsigned long long)mine) - 1u;
      mine &= mine - 1ull;
      if (live) out[c] = (uint16_t)(t0 + s);
      c += 1;
    }
  }
  return live ? c : 0u;
}

// Per-channel input spike-time lists, ascending, from the bitsets (steps
// 0 .. T-1); a wavefront per 64 channels.
template <typename real>
__global__ __launch_bounds__(256) void k_stage_in_lists(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= n.Iw) return;  // whole wavefronts
  const uint32_t i = w * 64 + lane_id();
  const bool live = i < n.I;
  uint16_t *out = n.spk_t + (size_t)b * n.spk_stride + (size_t)(live ? i : 0u) * n.Lc;
  const uint32_t c = column_lists(n.in_bits + (size_t)b * n.Tcap * n.Iw + w, n.Iw, 0, n.T[b], out, live);
  if (live) n.spk_cnt[(size_t)b * n.NS + i] = c;
}

// Spike-time lists of the recurrent neurons, ascending, from the bitsets of
// a finished forward pass (steps 1 .. T; the tiled forward kernel writes
// only the bitsets, so that a spike costs it no dependent global load); a
// wavefront per 64 neurons.
template <typename real>
__global__ __launch_bounds__(256) void k_stage_rec_lists(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= n.Jw) return;  // whole wavefronts
  const uint32_t j = w * 64 + lane_id();
  const bool live = j < n.J;
  uint16_t *out = n.spk_t + (size_t)b * n.spk_stride + (size_t)(n.I + (live ? j : 0u)) * n.Lc;
  const uint32_t c =
      column_lists(n.rec_bits + (size_t)b * (n.Tcap + 1) * n.Jw + w, n.Jw, 1, n.T[b] + 1, out, live);
  if (live) n.spk_cnt[(size_t)b * n.NS + n.I + j] = c;
}

// Teacher-forced recurrent spikes -> forced_bits[b][t][j].
template <typename real>
__global__ __launch_bounds__(256) void k_stage_forced(DevNet<real> n, uint32_t ntr, uint64_t nf) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += stride) {
    uint32_t lo = 0, hi = ntr;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (n.forced_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    const uint32_t t = n.forced_step[e], j = n.forced_neuron[e];
    if (t < 1 || t > n.T[lo] || j >= n.J) {
      atomicOr(&n.ctl[CTL_ERR], ERR_FORCED_RANGE);
      continue;
    }
    atomicOr((unsigned long long *)&n.forced_bits[((size_t)lo * (n.Tcap + 1) + t) * n.Jw + (j >> 6)],
             1ull << (j & 63u));
  }
}

// ----------------------------------------------------------------- forward

// One neuron update at step t (state in registers; the caller loads and
// stores it).  The expression order is that of the model definition, so the
// FP64 instantiation with an identically ordered input sum reproduces it bit
// for bit.  Writes psi; returns the spike.
template <typename real, bool FORCED>
__device__ inline bool neuron_step(const DevNet<real> &n, uint32_t b, uint32_t t, uint32_t j, bool live,
                                   real I, real beta, real &v, real &a, uint8_t &st) {
  uint32_t refr = st & 0x7Fu;
  const real zprev = (st & 0x80u) ? (real)1 : (real)0;
  real A = n.v_th;
  if (beta != (real)0) {  // LIF: v_th + 0 * a == v_th
    a = n.rho * a + zprev;
    A = n.v_th + beta * a;
  }
  if (n.reset_mode == 1) v = n.alpha * (zprev != (real)0 ? n.v_reset : v) + I;  // full reset to v_reset
  else v = n.alpha * v + I - zprev * A;
  const bool refractory = refr > 0;
  if (refractory) refr -= 1;
  bool z;
  if constexpr (FORCED) {
    const uint64_t fw = n.forced_bits[((size_t)b * (n.Tcap + 1) + t) * n.Jw + (j >> 6)];
    z = (fw >> (j & 63u)) & 1ull;
  } else {
    z = !refractory && v >= A;
  }
  z = z && live;
  const real ps = refractory ? (real)0 : surrogate(n, v - A);
  if (z) refr = n.n_ref;
  st = (uint8_t)(refr | (z ? 0x80u : 0u));
  n.psi[((size_t)b * (n.Tcap + 1) + t) * n.Jp + j] = ps;
  return z;
}

// Spike bitset word of this wavefront's 64 neurons and (LISTS) the
// spike-time list of each spiking neuron.  Called by whole wavefronts aligned
// to 64 neurons.
template <typename real, bool LISTS = true>
__device__ inline uint64_t publish_bits(const DevNet<real> &n, uint32_t b, uint32_t t, uint32_t j, bool z) {
  const uint64_t word = __ballot(z);
  if (lane_id() == 0) n.rec_bits[((size_t)b * (n.Tcap + 1) + t) * n.Jw + (j >> 6)] = word;
  if (LISTS && z) {
    const size_t ci = (size_t)b * n.NS + n.I + j;
    const uint32_t c = n.spk_cnt[ci];
    n.spk_t[(size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Lc + c] = (uint16_t)t;
    n.spk_cnt[ci] = c + 1;
  }
  return word;
}

// Exchange of the per-step spike lists between the tiles of a trial.  The
// word of a step-t entry carries t in its upper half, so a reader that sees
// the tag of step t sees that step's value: only the coherence of single
// locations is needed (system-scope atomic stores write through and
// system-scope atomic loads bypass the non-coherent caches), no fence and no
// barrier.  Double buffering by the parity of t is safe: a tile publishes
// step t+2 into the buffer of step t only after it has read every tile's
// step-t+1 list, and every tile publishes step t+1 only after it has read
// all step-t lists.  Waits are bounded; after the first timeout in the
// launch every wait returns at once and the batch reports an error.
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr uint32_t kMaxTiles = 1024;  // tiles per trial (at most one per thread of a tile workgroup)

__device__ inline uint64_t load_sys(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline void store_sys(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Queue event at p once its 16-bit tag (bits 48..63) is tag16, or 0 on
// timeout (flag ERR_SYNC): a zero event adds nothing.
__device__ inline uint64_t wait_event(const uint64_t *p, uint32_t tag16, uint32_t *err) {
  for (uint32_t spins = 0;; ++spins) {
    if ((spins & 255u) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_SYNC))
      return 0ull;
    if (spins > kSpinLimit) {
      atomicOr(err, ERR_SYNC);
      return 0ull;
    }
    __builtin_amdgcn_s_sleep(1);
    const uint64_t v = load_sys(p);
    if ((uint32_t)(v >> 48) == tag16) return v;
  }
}

// Low half of the step-t word at p, or 0 on timeout (flag ERR_SYNC).
__device__ inline uint32_t wait_tag(const uint64_t *p, uint32_t t, uint32_t *err) {
  uint64_t v = load_sys(p);
  if ((uint32_t)(v >> 32) == t) return (uint32_t)v;
  for (uint32_t spins = 0;; ++spins) {
    // first of all (and every 256 polls) give up if a wait of this batch already failed
    if ((spins & 255u) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_SYNC))
      return 0u;
    if (spins > kSpinLimit) {
      atomicOr(err, ERR_SYNC);
      return 0u;
    }
    __builtin_amdgcn_s_sleep(1);
    v = load_sys(p);
    if ((uint32_t)(v >> 32) == t) return (uint32_t)v;
  }
}

// Exclusive scan of one value per thread over the block (blockDim <= 1024);
// returns the prefix and writes the block total to *total.  wsum: LDS [17].
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t *wsum, uint32_t *total) {
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
    if ((int)lane >= o) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t i = 0; i < nw; ++i) {
      const uint32_t v = wsum[i];
      wsum[i] = acc;
      acc += v;
    }
    wsum[16] = acc;
  }
  __syncthreads();
  *total = wsum[16];
  return wsum[w] + inc - x;
}

// Delay-ring arithmetic.  FP32: fixed point with F fraction bits (weights
// rounded to nearest; the integer sums are exact); FP64: double.
struct RingScale {
  float to_fix;    // 2^F
  float from_fix;  // 2^-F
};

// F from the bound on |input current| per step: the largest F with
// l1max * 2^F <= 2^30, so that every partial sum and every rounding excess
// stays inside the int32 entry.  Below 8 fraction bits the bound is
// reported as an error.
__device__ inline RingScale ring_scale(const uint32_t *l1max, uint32_t *err) {
  constexpr int top = 30;
  const float l1 = __uint_as_float(*l1max);
  int F = top;
  if (l1 > 0.f) F = min(top, top - (int)ceilf(log2f(l1)));
  if (F < 8) {
    if (threadIdx.x == 0) atomicOr(err, ERR_INPUT_BOUND);
    F = max(F, -60);
  }
  return RingScale{ldexpf(1.f, F), ldexpf(1.f, -F)};
}

__device__ inline void ring_add(int32_t *p, float w, const RingScale &sc) {
  atomicAdd(p, __float2int_rn(w * sc.to_fix));
}
__device__ inline void ring_add(double *p, double w, const RingScale &) { atomicAdd(p, w); }
__device__ inline float ring_value(int32_t x, const RingScale &sc) { return (float)x * sc.from_fix; }
__device__ inline double ring_value(double x, const RingScale &) { return x; }

// Position of the r-th set bit of m (r < popcount(m)).
__device__ inline uint32_t nth_set_bit(uint64_t m, uint32_t r) {
  uint32_t pos = 0;
  for (uint32_t w = 32; w > 0; w >>= 1) {
    const uint64_t low = m & ((1ull << w) - 1ull);
    const uint32_t c = (uint32_t)__popcll(low);
    if (r >= c) {
      r -= c;
      m >>= w;
      pos += w;
    } else {
      m = low;
    }
  }
  return pos;
}

// Adds the spikes emitted at step t by inputs and by recurrent neurons of
// trial b into this tile's LDS ring.  Per chunk of up to 2 * blockDim
// spiking sources: every thread resolves two sources to their segments in
// the delivery table (the synapses of each source into this tile: weights,
// then ring offsets); segments are cut into pieces of P synapses, numbered
// by a block scan, and each source writes the entries of its pieces into
// the piece table.  A group of P consecutive lanes then takes one piece,
// one synapse per lane, so that a wavefront's loads cover a few contiguous
// lines; each group keeps U pieces in flight before adding the weights into
// the ring slots of their arrivals (only arrivals within the trial).  A
// lane's addresses come from one LDS read of its piece's entry.
// The segments of the step's input spikes of the first chunk are looked up
// before anything else (they do not depend on the other tiles).  The first
// E = 2 * blockDim / KT entries of every tile's list are read while the
// tiles' counts are awaited, and the segments of those already there are
// looked up at once, so that most recurrent sources of the first chunk are
// known without a further round trip; an entry whose tag is not yet there
// is awaited on its own.  Entries and segments are parked in the piece
// table, which the first chunk overwrites only after its last read of them.
// ptab: LDS [cap] (cap = n.ptab_cap >= 3 * blockDim); wsum: LDS [17].
// Piece entry: x = word index of the piece's first weight, y = synapse count
// | (distance from that weight to the piece's first ring offset, in uint16
// units) << 6.
// [P, U] of the delivery variants the autotuner chooses from; variant 0 is
// the default.  Variant 4 (FP32) delivers the spikes of steps 1.. through
// the per-tile queues instead (queue_spikes, drain_queues), and this
// function (kQueue) then delivers only the input spikes of step 0.
constexpr uint32_t kFwdVariants = 5;
constexpr uint32_t kNoEntry = 0xFFFFFFFFu;  // a parked list entry that had not arrived
constexpr uint32_t kQueueUnroll = 4;        // queue events a thread holds in flight
__host__ __device__ constexpr uint32_t fwd_piece(uint32_t v) { return v == 2 || v == 4 ? 4u : v == 3 ? 16u : 8u; }
__host__ __device__ constexpr uint32_t fwd_unroll(uint32_t) { return 8u; }
__host__ __device__ constexpr uint32_t fwd_rpt(uint32_t v) { return v == 1 || v == 2 ? 5u : 2u; }
__host__ __device__ constexpr bool fwd_queue(uint32_t v) { return v == 4; }

template <typename real, typename ring_t, uint32_t kPiece, uint32_t kUnroll, uint32_t kRpt, bool kQueue>
__device__ inline void deliver_tile(const DevNet<real> &n, uint32_t b, uint32_t k, uint32_t j0, uint32_t t,
                                    uint32_t Tb, ring_t *ring, const RingScale &sc,
                                    uint2 *ptab, uint32_t cap, uint32_t *wsum, const uint64_t *words,
                                    const uint32_t *woff, uint32_t nw, uint32_t own, uint32_t *tpre) {
  constexpr uint32_t WPR = sizeof(real) / 4;  // words per weight
  // parked entries [span] and their segments [span] (in the piece table)
  uint32_t *spec = reinterpret_cast<uint32_t *>(ptab);
  uint2 *spec_seg = ptab + (n.ptab_cap - blockDim.x * 2);
  const uint32_t span = 2 * blockDim.x;
  const uint32_t E = span / n.KT;  // >= 1: KT <= blockDim
  const uint64_t *isp = n.in_step_ptr + (size_t)b * (n.Tcap + 1);
  const uint64_t in_lo = isp[t], in_hi = isp[t + 1];
  const uint32_t n_in = in_hi > in_lo ? (uint32_t)(in_hi - in_lo) : 0u;
  const uint32_t *in_src = *reinterpret_cast<const uint32_t *const *>(n.ctl + CTL_WORDS);
  const uint32_t rk = tile_rank(k, n.KT);  // this tile's place in a source's dseg row
  uint2 iseg[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
#pragma unroll
  for (uint32_t u = 0; u < 2; ++u) {
    const uint32_t item = threadIdx.x + u * blockDim.x;
    if (item < n_in) iseg[u] = n.dseg[(size_t)in_src[in_lo + item] * n.KT + rk];
  }
  uint32_t n_rec = 0;
  const uint64_t *pl = n.pub_list + ((size_t)b * 2 + (t & 1u)) * n.Jp;
  // a single-tile trial takes its own spikes of the step (own of them) from
  // its LDS bitset words and their exclusive popcount prefix woff
  const bool local = n.KT == 1;
  if (t >= 1 && local) n_rec = own;
  if (!kQueue && t >= 1 && !local) {
    // the first E entries of every tile's list, read ahead of the counts
    uint64_t ahead[2] = {0ull, 0ull};
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      const uint32_t s = threadIdx.x + u * blockDim.x, tile = s / E, pos = s - tile * E;
      // (only inside the tile's part of the list buffer)
      if (tile < n.KT && pos < min(n.TS, n.Jp - tile * n.TS)) ahead[u] = load_sys(pl + (size_t)tile * n.TS + pos);
    }
    // segments of the entries already there
    uint2 aseg[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u)
      if ((uint32_t)(ahead[u] >> 32) == t)
        aseg[u] = n.dseg[(size_t)(n.I + min((uint32_t)ahead[u], n.J - 1u)) * n.KT + rk];
    // every tile's count of step t (published by the tiles, possibly still on the way)
    const uint32_t kk = threadIdx.x;
    uint32_t c = 0;
    if (kk < n.KT) {
      c = wait_tag(n.pub_cnt + ((size_t)b * 2 + (t & 1u)) * n.KT + kk, t, &n.ctl[CTL_ERR]);
      c = min(c, min(n.TS, n.Jp - kk * n.TS));
    }
    const uint32_t pre = block_exclusive_scan(c, wsum, &n_rec);
    if (kk < n.KT) tpre[kk] = pre;
    if (kk == 0) tpre[n.KT] = n_rec;
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      const uint32_t s = threadIdx.x + u * blockDim.x;
      if (s / E < n.KT) {
        const bool there = (uint32_t)(ahead[u] >> 32) == t;
        spec[s] = there ? (uint32_t)ahead[u] : kNoEntry;
        spec_seg[s] = aseg[u];
      }
    }
    __syncthreads();
  }
  const uint32_t total = n_in + n_rec;
  const uint32_t sbase = (t % n.R) * n.TS, RT = n.R * n.TS;
  // an arrival d steps later lies within the trial iff its ring offset is below lim
  const uint32_t lim = min(n.R, Tb - t + 1u) * n.TS;
  const uint32_t sub = threadIdx.x & (kPiece - 1u), grp = threadIdx.x / kPiece, ngrp = blockDim.x / kPiece;
  // chunks of kRpt * blockDim items, kRpt per thread
  for (uint32_t base = 0; base < total; base += kRpt * blockDim.x) {
    uint2 seg[kRpt];
    uint32_t src[kRpt];
    bool look[kRpt];  // segment still to be looked up
#pragma unroll
    for (uint32_t u = 0; u < kRpt; ++u) {
      seg[u] = make_uint2(0u, 0u);
      src[u] = 0u;
      look[u] = false;
    }
#pragma unroll
    for (uint32_t u = 0; u < kRpt; ++u) {
      const uint32_t item = base + threadIdx.x + u * blockDim.x;
      if (item >= total) continue;
      if (item < n_in) {
        if (base == 0 && u < 2) {
          seg[u] = iseg[u];
        } else {
          src[u] = in_src[in_lo + item];
          look[u] = true;
        }
        continue;
      }
      const uint32_t r = item - n_in;
      look[u] = true;
      if (local) {  // the r-th spike: word w with woff[w] <= r < woff[w + 1]
        uint32_t lw = 0, hw = nw;
        while (hw - lw > 1) {
          const uint32_t mid = (lw + hw) >> 1;
          if (woff[mid] <= r) lw = mid; else hw = mid;
        }
        const uint32_t jj = j0 + lw * 64 + nth_set_bit(words[lw], r - woff[lw]);
        src[u] = n.I + min(jj, n.J - 1u);
        continue;
      }
      uint32_t lk = 0, hk = n.KT;  // tpre[lk] <= r < tpre[hk]
      while (hk - lk > 1) {
        const uint32_t mid = (lk + hk) >> 1;
        if (tpre[mid] <= r) lk = mid; else hk = mid;
      }
      const uint32_t pos = r - tpre[lk];
      // parked entries are valid in the first chunk only (the piece table is reused after it)
      uint32_t j = base == 0 && pos < E ? spec[lk * E + pos] : kNoEntry;
      if (j != kNoEntry) {
        seg[u] = spec_seg[lk * E + pos];
        look[u] = false;
        continue;
      }
      j = wait_tag(pl + (size_t)lk * n.TS + pos, t, &n.ctl[CTL_ERR]);
      src[u] = n.I + min(j, n.J - 1u);
    }
#pragma unroll
    for (uint32_t u = 0; u < kRpt; ++u)
      if (look[u]) seg[u] = n.dseg[(size_t)src[u] * n.KT + rk];
    uint32_t np = 0;
#pragma unroll
    for (uint32_t u = 0; u < kRpt; ++u) np += (seg[u].y + kPiece - 1) / kPiece;
    uint32_t npieces;
    const uint32_t pre = block_exclusive_scan(np, wsum, &npieces);
    // (the scan's barrier also ends every read of the parked entries)
    for (uint32_t w0 = 0; w0 < npieces; w0 += cap) {
      const uint32_t w1 = min(npieces, w0 + cap);
      uint32_t p0 = pre;
#pragma unroll
      for (uint32_t u = 0; u < kRpt; ++u) {
        const uint32_t L = seg[u].y, nq = (L + kPiece - 1) / kPiece;
        for (uint32_t pc = max(p0, w0); pc < min(p0 + nq, w1); ++pc) {
          const uint32_t off = (pc - p0) * kPiece;
          const uint32_t dist = L * (sizeof(real) / 2) - off * (sizeof(real) / 2 - 1);
          ptab[pc - w0] = make_uint2(seg[u].x + off * WPR, min(kPiece, L - off) | (dist << 6));
        }
        p0 += nq;
      }
      __syncthreads();
      for (uint32_t pc0 = w0 + grp; pc0 < w1; pc0 += kUnroll * ngrp) {
        // branch-free address phase, then all loads, then the ring adds: the
        // loads of a group are in flight together (dead lanes read word 0 of
        // the table, which exists whenever there is a piece)
        uint32_t wi[kUnroll], oi[kUnroll];
        uint32_t live = 0;
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
          const uint32_t pc = pc0 + u * ngrp;
          const bool inb = pc < w1;
          const uint2 pe = ptab[inb ? pc - w0 : 0u];
          const bool ok = inb && sub < (pe.y & 63u);
          wi[u] = ok ? pe.x + sub * WPR : 0u;
          oi[u] = ok ? 2u * pe.x + (pe.y >> 6) + sub : 0u;
          live |= (uint32_t)ok << u;
        }
        real w[kUnroll];
        uint32_t o[kUnroll];
        const uint16_t *o16 = reinterpret_cast<const uint16_t *>(n.dlw);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
          w[u] = *reinterpret_cast<const real *>(n.dlw + wi[u]);
          o[u] = o16[oi[u]];
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
          if (!((live >> u) & 1u) || o[u] >= lim) continue;
          uint32_t ri = sbase + o[u];
          if (ri >= RT) ri -= RT;
          ring_add(&ring[ri], w[u], sc);
        }
      }
      __syncthreads();
    }
  }
}

// Recurrent part of a step with queues (FP32): one thread per source tile
// awaits that tile's count of step t for this tile in q_hdr, a block scan
// numbers the events, and every thread then takes kQueueUnroll events at a
// time: all their loads first, then any wait for an event whose tag has not
// arrived yet, then the ring additions (only arrivals within the trial).
// tpre: LDS [KT + 1]; qd: LDS [KT] starts of the regions into this tile.
__device__ inline void drain_queues(const DevNet<float> &n, uint32_t b, uint32_t k, uint32_t t, uint32_t Tb,
                                    int32_t *ring, const RingScale &sc, uint32_t *wsum, uint32_t *tpre,
                                    const uint32_t *qd, uint32_t tag) {
  const uint32_t KT = n.KT, kk = threadIdx.x;
  const size_t par = (size_t)b * 2 + (t & 1u);
  const uint64_t *hrow = n.q_hdr + (par * KT + k) * KT;
  const uint64_t *evq = n.q_ev + par * n.q_len;
  uint32_t c = 0;
  if (kk < KT) c = min(wait_tag(hrow + kk, tag, &n.ctl[CTL_ERR]), n.q_len - qd[kk]);
  uint32_t n_ev;
  const uint32_t pre = block_exclusive_scan(c, wsum, &n_ev);
  if (kk < KT) tpre[kk] = pre;
  if (kk == 0) tpre[KT] = n_ev;
  __syncthreads();
  const uint32_t tag16 = tag & 0xFFFFu;
  const uint32_t sbase = (t % n.R) * n.TS, RT = n.R * n.TS;
  const uint32_t lim = min(n.R, Tb - t + 1u) * n.TS;
  for (uint32_t r0 = threadIdx.x; r0 < n_ev; r0 += kQueueUnroll * blockDim.x) {
    uint32_t ad[kQueueUnroll];
    uint64_t ev[kQueueUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kQueueUnroll; ++u) {
      const uint32_t r = r0 + u * blockDim.x;
      ad[u] = kNoEntry;
      if (r < n_ev) {
        uint32_t lk = 0, hk = KT;  // tpre[lk] <= r < tpre[hk]
        while (hk - lk > 1) {
          const uint32_t mid = (lk + hk) >> 1;
          if (tpre[mid] <= r) lk = mid; else hk = mid;
        }
        ad[u] = qd[lk] + (r - tpre[lk]);
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kQueueUnroll; ++u) ev[u] = ad[u] != kNoEntry ? load_sys(evq + ad[u]) : 0ull;
#pragma unroll
    for (uint32_t u = 0; u < kQueueUnroll; ++u) {
      if (ad[u] == kNoEntry) continue;
      if ((uint32_t)(ev[u] >> 48) != tag16) ev[u] = wait_event(evq + ad[u], tag16, &n.ctl[CTL_ERR]);
      const uint32_t o = (uint32_t)(ev[u] >> 32) & 0xFFFFu;
      if (o >= lim) continue;
      uint32_t ri = sbase + o;
      if (ri >= RT) ri -= RT;
      ring_add(&ring[ri], __uint_as_float((uint32_t)ev[u]), sc);
    }
  }
}

// Source side of the queues (FP32): after the neuron update of step t, the
// tile copies the synapses of each of its spiking neurons into the queues
// of their target tiles, as tagged events, and of every input spike of step
// t the one segment into tile (k - i) mod KT (so each input spike is
// copied by all tiles together).  Per chunk of kQChunk items (the step's
// input spikes, then the tile's spikes), a thread takes its input's entry
// (those of the first chunk loaded before the neuron update: inz, iny) or finds
// its neuron from the bitset words and their popcount prefix, and a block
// scan numbers the items' non-empty segments (pp, pz).  Per batch of kQueueUnroll * blockDim segments, a thread takes
// kQueueUnroll of them and reserves each segment's place in the region
// (this tile -> target tile) with an LDS atomic on that tile's counter
// (bcnt; cst holds the counters at the start of the batch).  The batch's
// events are then staged in LDS ordered by target tile (bpl: the batch's
// prefix over target tiles) and flushed with consecutive lanes on
// consecutive places of a region, so that the write-through stores of a
// region's run combine (scattered 8-byte stores would each be a
// transaction of their own); batches larger than the staging array go in
// rounds.  Finally the counters go out as the step's q_hdr words and are
// cleared.  Every event carries its own tag, so a reader that sees a count
// does not depend on the order in which stores arrive.  The region
// (k -> kd) holds as many events as there are synapses from the tile's
// neurons to tile kd, and a neuron spikes at most once per step, so the
// reservations stay within it.
// pp, pz: LDS [kQChunk]; stg: LDS [scap]; bcnt, qs, cst: LDS [KT]; bpl: LDS [KT + 1].
constexpr uint32_t kQChunk = 256;
__device__ inline void queue_spikes(const DevNet<float> &n, uint32_t b, uint32_t k, uint32_t j0, uint32_t t,
                                    uint32_t tag, const uint64_t *words, const uint32_t *woff, uint32_t nw,
                                    uint32_t gtot, uint64_t in_lo, uint32_t n_in, uint32_t inz, uint32_t iny,
                                    uint32_t *pp,
                                    uint32_t *pz, uint2 *stg, uint32_t scap, uint32_t *bcnt, const uint32_t *qs,
                                    uint32_t *cst, uint32_t *bpl, uint32_t *wsum) {
  const uint32_t KT = n.KT;
  const size_t par = (size_t)b * 2 + (t & 1u);
  uint64_t *evq = n.q_ev + par * n.q_len;
  const uint64_t hi = (uint64_t)(tag & 0xFFFFu) << 48;
  const uint16_t *o16 = reinterpret_cast<const uint16_t *>(n.dlw);
  const uint32_t *in_src = *reinterpret_cast<const uint32_t *const *>(n.ctl + CTL_WORDS);
  const uint32_t items = n_in + gtot;
  for (uint32_t c0 = 0; c0 < items; c0 += kQChunk) {
    const uint32_t r = c0 + threadIdx.x;
    uint32_t np = 0, z0 = 0;
    if (threadIdx.x < kQChunk && r < items) {
      if (r >= n_in) {  // the (r - n_in)-th spike: word lw with woff[lw] <= r - n_in < woff[lw + 1]
        const uint32_t rr = r - n_in;
        uint32_t lw = 0, hw = nw;
        while (hw - lw > 1) {
          const uint32_t mid = (lw + hw) >> 1;
          if (woff[mid] <= rr) lw = mid; else hw = mid;
        }
        const uint32_t j = min(j0 + lw * 64 + nth_set_bit(words[lw], rr - woff[lw]), n.J - 1u);
        z0 = n.q_nzp[j];
        np = n.q_nzp[j + 1] - z0;
      } else {
        z0 = c0 == 0 ? inz : n.q_in + min(in_src[in_lo + r], n.I - 1u) * KT + k;
        np = ((c0 == 0 ? iny : n.q_nz[z0].y) & 0xFFFFu) ? 1u : 0u;
      }
    }
    uint32_t npairs;
    const uint32_t pre = block_exclusive_scan(np, wsum, &npairs);
    if (threadIdx.x < kQChunk) {
      pp[threadIdx.x] = pre;
      pz[threadIdx.x] = z0;
    }
    for (uint32_t kd = threadIdx.x; kd < KT; kd += blockDim.x) cst[kd] = bcnt[kd];
    __syncthreads();
    const uint32_t nown = min(kQChunk, items - c0);
    for (uint32_t s0 = 0; s0 < npairs; s0 += kQueueUnroll * blockDim.x) {
      uint2 ent[kQueueUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kQueueUnroll; ++u) {
        const uint32_t p = s0 + u * blockDim.x + threadIdx.x;
        ent[u] = make_uint2(0u, 0u);
        if (p < npairs) {
          uint32_t lo = 0, hs = nown;  // pp[lo] <= p < pp[lo + 1]
          while (hs - lo > 1) {
            const uint32_t mid = (lo + hs) >> 1;
            if (pp[mid] <= p) lo = mid; else hs = mid;
          }
          ent[u] = n.q_nz[pz[lo] + (p - pp[lo])];
        }
      }
      // the first two synapses of every segment, loaded before anything waits for them
      uint32_t w2[kQueueUnroll][2], o2[kQueueUnroll][2];
#pragma unroll
      for (uint32_t u = 0; u < kQueueUnroll; ++u) {
        const uint32_t L = ent[u].y & 0xFFFFu;
#pragma unroll
        for (uint32_t i = 0; i < 2; ++i) {
          w2[u][i] = i < L ? n.dlw[ent[u].x + i] : 0u;
          o2[u][i] = i < L ? o16[2u * (ent[u].x + L) + i] : 0u;
        }
      }
      uint32_t rel[kQueueUnroll];  // place in the region, relative to the batch's start
#pragma unroll
      for (uint32_t u = 0; u < kQueueUnroll; ++u) {
        const uint32_t L = ent[u].y & 0xFFFFu, kd = ent[u].y >> 16;
        rel[u] = L ? atomicAdd(&bcnt[kd], L) - cst[kd] : 0u;
      }
      __syncthreads();
      uint32_t cb = 0;
      if (threadIdx.x < KT) cb = bcnt[threadIdx.x] - cst[threadIdx.x];
      uint32_t nev;
      const uint32_t bpre = block_exclusive_scan(cb, wsum, &nev);
      if (threadIdx.x < KT) bpl[threadIdx.x] = bpre;
      if (threadIdx.x == 0) bpl[KT] = nev;
      __syncthreads();
      uint32_t bp[kQueueUnroll];  // batch position of each segment's first event
#pragma unroll
      for (uint32_t u = 0; u < kQueueUnroll; ++u) bp[u] = (ent[u].y & 0xFFFFu) ? bpl[ent[u].y >> 16] + rel[u] : 0u;
      for (uint32_t r0 = 0; r0 < nev; r0 += scap) {
        const uint32_t r1 = min(nev, r0 + scap);
#pragma unroll
        for (uint32_t u = 0; u < kQueueUnroll; ++u) {
          const uint32_t L = ent[u].y & 0xFFFFu;
          const uint32_t i0 = bp[u] < r0 ? r0 - bp[u] : 0u;
          const uint32_t i1 = min(L, r1 > bp[u] ? r1 - bp[u] : 0u);
          for (uint32_t i = i0; i < i1; ++i) {
            uint2 v;
            if (i < 2) {
              v = make_uint2(i == 0 ? w2[u][0] : w2[u][1], i == 0 ? o2[u][0] : o2[u][1]);
            } else {
              v = make_uint2(n.dlw[ent[u].x + i], o16[2u * (ent[u].x + L) + i]);
            }
            stg[bp[u] + i - r0] = v;
          }
        }
        __syncthreads();
        for (uint32_t e = r0 + threadIdx.x; e < r1; e += blockDim.x) {
          uint32_t lk = 0, hk = KT;  // bpl[lk] <= e < bpl[hk]
          while (hk - lk > 1) {
            const uint32_t mid = (lk + hk) >> 1;
            if (bpl[mid] <= e) lk = mid; else hk = mid;
          }
          const uint2 v = stg[e - r0];
          store_sys(evq + qs[lk] + cst[lk] + (e - bpl[lk]), hi | (uint64_t)v.y << 32 | v.x);
        }
        __syncthreads();
      }
      for (uint32_t kd = threadIdx.x; kd < KT; kd += blockDim.x) cst[kd] = bcnt[kd];
      __syncthreads();
    }
  }
  for (uint32_t kd = threadIdx.x; kd < KT; kd += blockDim.x) {
    const uint32_t c = bcnt[kd];
    bcnt[kd] = 0u;
    store_sys(n.q_hdr + (par * KT + kd) * KT + k, (uint64_t)tag << 32 | c);
  }
}

// Persistent forward pass over steps ctl[T0]+1 .. ctl[T0]+nsteps of trials
// b0 .. b0 + gridDim.x / KT - 1.  Workgroup (b, k) owns neurons
// [k*TS, k*TS + TS) of trial b; their delay ring and
// state stay in LDS for the whole launch.  Per step: neuron update of the
// tile, spike publication (bitset, spike times, the tile's tagged spike list
// and count), then delivery of all tiles' spikes of the step into the
// tile's ring, reading each tile's list as soon as its tag shows up.  With
// the queue variant (Q) the tile instead copies its spikes' synapses, and
// its share of the input spikes', into the per-tile queues, then drains its
// own queues.  The KT workgroups of a trial must be resident together
// (checked on the host).
template <typename real, typename ring_t, bool FORCED, uint32_t VAR>
__global__ __launch_bounds__(1024) void k_forward_tiled(DevNet<real> n, uint32_t nsteps, uint32_t b0) {
  constexpr uint32_t P = fwd_piece(VAR), U = fwd_unroll(VAR), RPT = fwd_rpt(VAR);
  constexpr bool Q = fwd_queue(VAR) && sizeof(real) == 4;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t KT = n.KT, TS = n.TS;
  const uint32_t bl = blockIdx.x / KT, k = blockIdx.x - bl * KT, b = b0 + bl;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t Tb = n.T[b];
  const uint32_t t0 = n.ctl[CTL_T0];
  if (t0 >= Tb) return;  // the same for every workgroup of the trial
  const uint32_t j0 = k * TS;
  const uint32_t nt = min(TS, n.Jp - j0);  // multiple of 64
  const uint32_t nw = nt >> 6;
  ring_t *ring = reinterpret_cast<ring_t *>(smem);
  ring_t *gring = static_cast<ring_t *>(n.ring);
  real *sv = reinterpret_cast<real *>(ring + (size_t)n.R * TS);
  real *sa = sv + TS;
  uint64_t *words = reinterpret_cast<uint64_t *>(sa + TS);
  uint32_t *woff = reinterpret_cast<uint32_t *>(words + TS / 64);
  uint2 *ptab = reinterpret_cast<uint2 *>(woff + ((TS / 64 + 2) & ~1u));  // 8-byte aligned
  uint8_t *sst = reinterpret_cast<uint8_t *>(ptab + n.ptab_cap);
  uint64_t *salif = reinterpret_cast<uint64_t *>(sst + TS);  // [TS / 64] ALIF neurons of the tile
  __shared__ uint32_t gtot;
  __shared__ uint32_t wsum[17];
  __shared__ uint32_t tpre[kMaxTiles + 1];  // prefix of the tiles' spike (or queue event) counts of a step
  // queues: the piece table's last 5 * KT + 2 words hold the tile's
  // per-target-tile counters, region starts (as a source, qs; as a target,
  // qd) and the source side's batch arrays cst, bpl; the rest serves the
  // input deliveries' pieces and, on the source side, the chunk arrays pp,
  // pz [kQChunk] followed by the staging array stg [scap]
  uint32_t *pu = reinterpret_cast<uint32_t *>(ptab);
  uint32_t pcap = n.ptab_cap, scap = 0, tag0 = 0;
  uint32_t *bcnt = nullptr, *qs = nullptr, *qd = nullptr, *cst = nullptr, *bpl = nullptr;
  uint2 *stg = nullptr;
  if constexpr (Q) {
    const uint32_t tail = 5 * KT + 2;
    bcnt = pu + 2 * n.ptab_cap - tail;
    qs = bcnt + KT;
    qd = qs + KT;
    cst = qd + KT;
    bpl = cst + KT;
    pcap = (2 * n.ptab_cap - tail) / 2;
    scap = (2 * n.ptab_cap - 2 * kQChunk - tail) / 2;
    stg = reinterpret_cast<uint2 *>(pu + 2 * kQChunk);
    tag0 = n.ctl[CTL_TAG0];
    for (uint32_t i = threadIdx.x; i < KT; i += blockDim.x) {
      bcnt[i] = 0u;
      qs[i] = n.q_src[(size_t)k * KT + i];
      qd[i] = n.q_dst[(size_t)k * KT + i];
    }
  }
  RingScale sc{1.f, 1.f};
  if constexpr (sizeof(real) == 4) sc = ring_scale(n.l1max, &n.ctl[CTL_ERR]);

  const size_t gs = (size_t)b * n.Jp + j0;
  for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) {
    sv[i] = n.v[gs + i];
    sa[i] = n.a[gs + i];
    sst[i] = n.nst[gs + i];
    for (uint32_t r = 0; r < n.R; ++r) ring[r * TS + i] = gring[((size_t)b * n.R + r) * n.Jp + j0 + i];
    const uint64_t m = __ballot(n.any_alif && n.beta_j[j0 + i] != (real)0);
    if (lane_id() == 0) salif[i >> 6] = m;
  }
  __syncthreads();
  if (t0 == 0) {  // inputs emitted at step 0
    deliver_tile<real, ring_t, P, U, RPT, Q>(n, b, k, j0, 0, Tb, ring, sc, ptab, pcap, wsum, words, woff, 0u, 0u,
                                             tpre);
    __syncthreads();
  }
  const uint32_t t_end = min(t0 + nsteps, Tb);
  for (uint32_t t = t0 + 1; t <= t_end; ++t) {
    const uint32_t slot = t % n.R;
    // queues: the step's input spikes, and the entry of the first kQChunk of
    // them, loaded before the neuron update
    uint64_t in_lo = 0;
    uint32_t n_in = 0, inz = 0, iny = 0;
    if constexpr (Q) {
      const uint64_t *isp = n.in_step_ptr + (size_t)b * (n.Tcap + 1);
      in_lo = isp[t];
      const uint64_t in_hi = t < Tb ? isp[t + 1] : in_lo;
      n_in = in_hi > in_lo ? (uint32_t)(in_hi - in_lo) : 0u;
      if (threadIdx.x < min(n_in, kQChunk)) {
        const uint32_t *in_src = *reinterpret_cast<const uint32_t *const *>(n.ctl + CTL_WORDS);
        inz = n.q_in + min(in_src[in_lo + threadIdx.x], n.I - 1u) * KT + k;
        iny = n.q_nz[inz].y;
      }
    }
    for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) {
      real v = sv[i], a = sa[i];
      uint8_t st = sst[i];
      const real I = ring_value(ring[slot * TS + i], sc);
      ring[slot * TS + i] = (ring_t)0;
      const uint32_t j = j0 + i;
      const real beta = (salif[i >> 6] >> (i & 63u)) & 1ull ? n.beta_a : (real)0;
      const bool z = neuron_step<real, FORCED>(n, b, t, j, j < n.J, I, beta, v, a, st);
      sv[i] = v;
      sa[i] = a;
      sst[i] = st;
      const uint64_t word = publish_bits<real, false>(n, b, t, j, z);
      if (lane_id() == 0) words[i >> 6] = word;
    }
    __syncthreads();
    // compacted spike list of the tile: one wavefront scans the tile's words
    if (threadIdx.x < 64) {
      uint32_t off = 0, tot = 0;
      for (uint32_t w0 = 0; w0 < nw; w0 += 64) {
        const uint32_t w = w0 + threadIdx.x;
        const uint32_t c = w < nw ? (uint32_t)__popcll(words[w]) : 0u;
        uint32_t inc = c;  // inclusive scan across the wavefront
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
          if ((int)threadIdx.x >= o) inc += y;
        }
        if (w < nw) woff[w] = off + inc - c;
        off += (uint32_t)__shfl((int)inc, 63);
      }
      tot = off;
      if (threadIdx.x == 0) gtot = tot;
    }
    __syncthreads();
    if constexpr (Q) {
      if (t < Tb) {
        queue_spikes(n, b, k, j0, t, tag0 + t, words, woff, nw, gtot, in_lo, n_in, inz, iny, pu, pu + kQChunk, stg,
                     scap, bcnt, qs, cst, bpl, wsum);
        drain_queues(n, b, k, t, Tb, ring, sc, wsum, tpre, qd, tag0 + t);
      }
    } else if (KT > 1) {  // publish the tile's spikes of step t: the entries, then the count
      // (a single-tile trial delivers its spikes from its own LDS bitset)
      uint64_t *pl = n.pub_list + ((size_t)b * 2 + (t & 1u)) * n.Jp + j0;
      const uint64_t tag = (uint64_t)t << 32;
      for (uint32_t w = threadIdx.x >> 6; w < nw; w += blockDim.x >> 6) {
        const uint64_t word = words[w];
        const uint32_t lane = lane_id();
        if ((word >> lane) & 1ull)
          store_sys(&pl[woff[w] + (uint32_t)__popcll(word & ((1ull << lane) - 1ull))], tag | (j0 + w * 64 + lane));
      }
      __syncthreads();
      if (threadIdx.x == 0) store_sys(&n.pub_cnt[((size_t)b * 2 + (t & 1u)) * KT + k], tag | gtot);
    }
    if (!Q && t < Tb)
      deliver_tile<real, ring_t, P, U, RPT, Q>(n, b, k, j0, t, Tb, ring, sc, ptab, pcap, wsum, words, woff, nw, gtot,
                                               tpre);
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) {
    n.v[gs + i] = sv[i];
    n.a[gs + i] = sa[i];
    n.nst[gs + i] = sst[i];
    for (uint32_t r = 0; r < n.R; ++r) gring[((size_t)b * n.R + r) * n.Jp + j0 + i] = ring[r * TS + i];
  }
}

// Deterministic per-step neuron update: every target sums its arriving
// synapses in ascending source order, inputs first (the reference order).
template <typename real, bool FORCED>
__global__ __launch_bounds__(256) void k_neuron_gather(DevNet<real> n, uint32_t off) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t t = n.ctl[CTL_T0] + off;
  const uint32_t Tb = n.T[b];
  if (t == 0 || t > Tb) return;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n.Jp) return;  // whole wavefronts: Jp is a multiple of 64
  const bool live = j < n.J;
  const size_t sidx = (size_t)b * n.Jp + j;
  real I = 0;
  if (live) {
    const uint64_t *inb = n.in_bits + (size_t)b * n.Tcap * n.Iw;
    const uint64_t *rb = n.rec_bits + (size_t)b * (n.Tcap + 1) * n.Jw;
    const uint32_t q1 = n.tm_ptr[j + 1];
    for (uint32_t q = n.tm_ptr[j]; q < q1; ++q) {
      const uint32_t pk = n.tm_syn[q];
      const uint32_t src = pk & 0xFFFFFFu;
      const int s = (int)t - (int)(pk >> 24);
      bool hit;
      if (src < n.I) {
        hit = s >= 0 && ((inb[(size_t)s * n.Iw + (src >> 6)] >> (src & 63u)) & 1ull);
      } else {
        const uint32_t r = src - n.I;
        hit = s >= 1 && ((rb[(size_t)s * n.Jw + (r >> 6)] >> (r & 63u)) & 1ull);
      }
      if (hit) I = I + n.tm_w[q];
    }
  }
  real v = n.v[sidx], a = n.a[sidx];
  uint8_t st = n.nst[sidx];
  const bool z = neuron_step<real, FORCED>(n, b, t, j, live, I, n.beta_j[j], v, a, st);
  n.v[sidx] = v;
  n.a[sidx] = a;
  n.nst[sidx] = st;
  publish_bits(n, b, t, j, z);
}

__global__ void k_advance(uint32_t *ctl, uint32_t by) {
  if (threadIdx.x == 0) ctl[CTL_T0] += by;
}

// ----------------------------------------------------------------- readout

// ysum[b][t][k] = sum over neurons j spiking at t of W_out[k][j] (FP64),
// one wavefront per (trial, step), fixed reduction order.
template <typename real>
__global__ __launch_bounds__(256) void k_readout_sums(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6) + 1;
  if (t > n.T[b]) return;
  const uint32_t lane = lane_id();
  const uint64_t *row = n.rec_bits + ((size_t)b * (n.Tcap + 1) + t) * n.Jw;
  double *out = n.ysum + ((size_t)b * (n.Tcap + 2) + t) * n.K;
  uint32_t nsp = 0;
  for (uint32_t w = lane; w < n.Jw; w += 64) nsp += (uint32_t)__popcll(row[w]);
  for (int o = 32; o > 0; o >>= 1) nsp += (uint32_t)__shfl_down((int)nsp, o);
  if (lane == 0) n.nspk[(size_t)b * (n.Tcap + 1) + t] = nsp;
  for (uint32_t k0 = 0; k0 < n.K; k0 += 8) {
    double acc[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0;
    for (uint32_t w = lane; w < n.Jw; w += 64) {
      uint64_t word = row[w];
      while (word) {
        const uint32_t j = w * 64 + (uint32_t)(__ffsll((unsigned long long)word) - 1);
        word &= word - 1ull;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (k0 + kk < n.K) acc[kk] += (double)n.w_out[(size_t)(k0 + kk) * n.Jp + j];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      for (int o = 32; o > 0; o >>= 1) acc[kk] += __shfl_down(acc[kk], o);
    if (lane == 0)
      for (int kk = 0; kk < 8; ++kk)
        if (k0 + kk < n.K) out[k0 + kk] = acc[kk];
  }
}

// Per trial (one block of 256): readout recursion y^t = kappa y^{t-1} +
// ysum^{t-d} (readout delay d, Supplementary "Delay from the recurrent to the
// output layer"), error signal and loss (window-gated; MSE, cross-entropy
// or temporal MSE), the rate regulariser's loss (static or moving average),
// prediction, and the backward filters of the error shifted by d:
// ebar^u = E^{u+d} + kappa_e ebar^{u+1} up to u = T-d-d^ls (the learning
// signals the recurrent gradient takes, with the eligibility's filter) and
// ebo^u with kappa up to u = T-d (output gradient); both 0 beyond.  All
// FP64, fixed summation order.
template <typename real>
__global__ __launch_bounds__(256) void k_readout_scan(DevNet<real> n) {
  const uint32_t b = blockIdx.x;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t T = n.T[b], K = n.K, tid = threadIdx.x, d = n.d_out;
  const size_t rs = (size_t)(n.Tcap + 2) * K;
  double *ysum = n.ysum + b * rs, *y = n.y + b * rs, *err = n.err + b * rs, *ebar = n.ebar + b * rs;
  double *ebo = n.ebo + b * rs;
  const double kap = n.kappa_d;
  // the serial scans below take their inputs 16 steps at a time, loaded
  // before the recursion needs them, so that a step does not wait for memory
  for (uint32_t k = tid; k < K; k += blockDim.x) {
    double yy = 0.0;
    for (uint32_t t0 = 1; t0 <= T; t0 += 16) {
      double in[16];
#pragma unroll
      for (uint32_t u = 0; u < 16; ++u) {
        const uint32_t t = t0 + u;
        in[u] = (t <= T && t > d) ? ysum[(size_t)(t - d) * K + k] : 0.0;
      }
#pragma unroll
      for (uint32_t u = 0; u < 16; ++u) {
        const uint32_t t = t0 + u;
        if (t <= T) {
          yy = kap * yy + in[u];
          y[(size_t)t * K + k] = yy;
        }
      }
    }
  }
  __syncthreads();
  double lp = 0.0;
  const uint32_t label = n.loss != 0 ? n.label[b] : 0u;
  for (uint32_t t = 1 + tid; t <= T; t += blockDim.x) {
    const bool win = n.window ? n.window[(size_t)b * n.step_stride + t - 1] != 0 : true;
    const double *yt = y + (size_t)t * K;
    double *et = err + (size_t)t * K;
    if (n.loss == 0) {
      const double *tg = n.target + ((size_t)b * n.step_stride + t - 1) * K;
      for (uint32_t k = 0; k < K; ++k) {
        const double d = yt[k] - tg[k];
        et[k] = win ? d : 0.0;
        if (win) lp += 0.5 * d * d;
      }
    } else if (n.loss == 2) {
      // eq. temporal-mse on the one-hot label; the window's y rows (kept in
      // the ysum row, no longer needed) give the prediction
      double *yw = ysum + (size_t)t * K;
      for (uint32_t k = 0; k < K; ++k) {
        const double d = yt[k] - (k == label ? 1.0 : 0.0);
        et[k] = win ? 2.0 / K * d : 0.0;
        if (win) lp += d * d / K;
        yw[k] = win ? yt[k] : 0.0;
      }
    } else {
      double mx = yt[0];
      for (uint32_t k = 1; k < K; ++k) mx = fmax(mx, yt[k]);
      double se = 0.0;
      for (uint32_t k = 0; k < K; ++k) se += exp(yt[k] - mx);
      double *pi_t = ysum + (size_t)t * K;  // ysum row no longer needed: keep window-gated pi
      for (uint32_t k = 0; k < K; ++k) {
        const double pi = exp(yt[k] - mx) / se;
        et[k] = win ? pi - (k == label ? 1.0 : 0.0) : 0.0;
        pi_t[k] = win ? pi : 0.0;
      }
      if (win) lp += -(yt[label] - mx - log(se));
    }
  }
  if (n.c_reg != 0.0 && n.reg_mode == 0) {
    const uint32_t *cnt = n.spk_cnt + (size_t)b * n.NS + n.I;
    double rl = 0.0;
    for (uint32_t j = tid; j < n.J; j += blockDim.x) {
      const double f = (double)cnt[j] / (double)T - n.f_target;
      rl += f * f;
    }
    lp += 0.5 * n.c_reg * rl;
  } else if (n.c_reg != 0.0) {
    // moving-average rate (eq. ema-rate) of each neuron, step by step from
    // its spike times; loss c/2 sum_t (f^t - f*)^2, each neuron's sum first
    const double be = n.beta_f, fs = n.f_target;
    double rl = 0.0;
    for (uint32_t j = tid; j < n.J; j += blockDim.x) {
      const uint32_t c = n.spk_cnt[(size_t)b * n.NS + n.I + j];
      const uint16_t *st = n.spk_t + (size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Lc;
      double f = 0.0, sj = 0.0;
      uint32_t i = 0;
      for (uint32_t t = 1; t <= T; ++t) {
        double z = 0.0;
        if (i < c && st[i] == t) {
          z = 1.0;
          ++i;
        }
        f = be * f + (1.0 - be) * z;
        const double df = f - fs;
        sj += df * df;
      }
      rl += 0.5 * n.c_reg * sj;
    }
    lp += rl;
  }
  __shared__ double red[256];
  __shared__ double psum[64];
  red[tid] = lp;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  // last index of each filter (signed: a trial may be shorter than the delays)
  const int64_t u_out = (int64_t)T - d, u_rec = u_out - (int64_t)n.d_ls;
  const double kap_e = n.kappa_e_d;
  for (uint32_t k = tid; k < K; k += blockDim.x) {
    double eb = 0.0, eo = 0.0;
    for (int64_t u0 = T; u0 >= 1; u0 -= 16) {
      double in[16];
#pragma unroll
      for (int64_t q = 0; q < 16; ++q) {
        const int64_t u = u0 - q;
        in[q] = (u >= 1 && u <= u_out) ? err[(size_t)(u + d) * K + k] : 0.0;
      }
#pragma unroll
      for (int64_t q = 0; q < 16; ++q) {
        const int64_t u = u0 - q;
        if (u >= 1) {
          const double e = in[q];
          eo = e + kap * eo;
          eb = u <= u_rec ? e + kap_e * eb : 0.0;
          ebar[(size_t)u * K + k] = eb;
          if (ebo != ebar) ebo[(size_t)u * K + k] = eo;
        }
      }
    }
    if (n.loss != 0 && k < 64) {
      double s = 0.0;
      for (uint32_t t0 = 1; t0 <= T; t0 += 16) {
        double in[16];
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) in[u] = t0 + u <= T ? ysum[(size_t)(t0 + u) * K + k] : 0.0;
#pragma unroll
        for (uint32_t u = 0; u < 16; ++u) s += in[u];
      }
      psum[k] = s;
    }
  }
  {
    unsigned long long ns = 0;
    for (uint32_t t = 1 + tid; t <= T; t += blockDim.x) ns += n.nspk[(size_t)b * (n.Tcap + 1) + t];
    if (ns) atomicAdd(&n.cnt[CNT_REC_SPIKES], ns);
  }
  __syncthreads();
  if (tid == 0) {
    n.loss_out[b] = red[0];
    uint32_t best = 0;
    if (n.loss != 0)
      for (uint32_t k = 1; k < K && k < 64; ++k)
        if (psum[k] > psum[best]) best = k;
    n.pred_out[b] = best;
  }
}

// ----------------------------------------------------------------- gradient

// Per (trial, neuron), backward over the trial in chunks of 16 steps:
// learning signal of the filtered errors Lambda^t = sum_k B_jk Ebar_k^t (plus
// the rate regulariser's constant for t <= T - d), the adjoint recursion of the eligibility vector (FP64) and the archive
// phi[b][j][t] = mu^t[0]; then the neuron's output-synapse gradient
// sum over its spikes u of Ebar_k^u (without the learning-signal cut).  B rows and the chunk's Ebar rows are
// read from LDS; phi is transposed through LDS so that each store writes
// whole 16-step row segments.
// PLUS: the full reset or the moving-average regulariser is on (compiled
// out otherwise, so the plain form keeps its registers).
template <typename real, bool PLUS>
__global__ __launch_bounds__(256) void k_adjoint(DevNet<real> n) {
  extern __shared__ __align__(16) unsigned char adj_smem[];
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  const uint32_t j = blockIdx.x * bd + tid;
  const uint32_t T = n.T[b], K = n.K;
  const bool live = j < n.J;
  const bool inrow = j < n.Jp;
  double *fbl = reinterpret_cast<double *>(adj_smem);   // [K][bd]
  double *ebl = fbl + (size_t)K * bd;                   // [K][16]
  real *tile = reinterpret_cast<real *>(ebl + 16 * K);  // [bd][17]
  for (uint32_t k = 0; k < K; ++k) fbl[k * bd + tid] = live ? (double)n.fb[(size_t)j * K + k] : 0.0;
  const double beta = live ? (double)n.beta_j[j] : 0.0;
  const double *eb = n.ebar + (size_t)b * (n.Tcap + 2) * K;
  // rate regulariser (eq. firing-rate-regularization): c^reg/T (f_j - f*)
  // multiplies the eligibility of every step u <= T - d, so it adds to the
  // adjoint's learning-signal sum there
  const bool ema = PLUS && n.reg_mode == 1;
  const double creg = (live && n.c_reg != 0.0 && !ema)
                          ? n.c_reg / (double)T *
                                ((double)n.spk_cnt[(size_t)b * n.NS + n.I + j] / (double)T - n.f_target)
                          : 0.0;
  const int64_t u_reg = (int64_t)T - n.d_out;
  const uint32_t wbase = tid & ~63u, lane = tid & 63u;
  const uint32_t c = live ? n.spk_cnt[(size_t)b * n.NS + n.I + j] : 0u;
  const uint16_t *st = n.spk_t + (size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Lc;
  real *phi_row = n.phi + ((size_t)b * n.Jp + j) * n.Tp;
  // Moving-average regulariser (eq. ema-gradient): sum_s c (f^s - f*) G_beta(e^s)
  // over s <= T - d equals sum_s e^s R^s with the backward filter
  // R^s = c (1 - beta)(f^s - f*) + beta R^{s+1}, added to the learning-signal
  // sum.  The rate f (eq. ema-rate) is f^u at the neuron's spike steps u and
  // decays by beta in between; its values at the spikes are computed forward
  // first and parked in the neuron's archive row at those steps, which the
  // backward pass overwrites only after it has read them.
  if constexpr (PLUS) {
    if (ema && live) {
      double f = 0.0;
      uint32_t prev = 0;
      for (uint32_t i = 0; i < c; ++i) {
        f = n.beta_f * f * pow(n.beta_f, (double)(st[i] - prev - 1)) + (1.0 - n.beta_f);
        prev = st[i];
        phi_row[st[i]] = (real)f;
      }
    }
  }
  int32_t sp_i = (int32_t)c - 1;  // last spike at or before the current step
  double f_sp = (ema && sp_i >= 0) ? (double)phi_row[st[sp_i]] : 0.0, R = 0.0;
  const uint64_t *zrow = n.rec_bits + (size_t)b * (n.Tcap + 1) * n.Jw + (inrow ? (j >> 6) : 0u);
  double mu0 = 0.0, mu1 = 0.0;
  // The psi rows and error values of a chunk are loaded one chunk ahead,
  // before the archive stores of the current chunk: vector memory operations
  // complete in order on this GPU, so a load issued after those stores would
  // wait for them.  (Error values ahead only while they fit 4 per thread.)
  const bool e_ahead = 16 * K <= 4 * bd;
  real psn[16];
  double en[4];
  // branch-free, with no use of the values until the next chunk: every lane
  // loads from a clamped, valid address, and what lies outside the trial is
  // dropped where the values are used
  const real *ps_safe = n.psi + (size_t)b * (n.Tcap + 1) * n.Jp + (inrow ? j : 0u);
  auto fetch = [&](uint32_t tc) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t t = tc + r, tt = t < 1 ? 1u : (t > T ? T : t);
      psn[r] = ps_safe[(size_t)tt * n.Jp];
    }
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t idx = tid + q * bd, k = idx >> 4, t = tc + (idx & 15u);
      const bool ok = e_ahead && idx < 16 * K && t >= 1 && t <= T;
      en[q] = eb[ok ? (size_t)t * K + k : 0u];
    }
  };
  fetch((T / 16) * 16);
  for (int m = (int)(T / 16); m >= 0; --m) {
    const uint32_t tb = (uint32_t)m * 16;
    real ps[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) ps[r] = psn[r];
    __syncthreads();
    if (e_ahead) {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t idx = tid + q * bd, t = tb + (idx & 15u);
        if (idx < 16 * K) ebl[idx] = (t >= 1 && t <= T) ? en[q] : 0.0;
      }
    } else {
      for (uint32_t idx = tid; idx < 16 * K; idx += bd) {
        const uint32_t k = idx >> 4, t = tb + (idx & 15u);
        ebl[idx] = (t >= 1 && t <= T) ? eb[(size_t)t * K + k] : 0.0;
      }
    }
    if (m > 0) fetch(tb - 16);
    __syncthreads();
    // Lambda of the chunk's 16 steps: k outer, so each B_jk is read once per
    // chunk and the 16 error values of k are one broadcast row
    double lam[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) lam[r] = 0.0;
    for (uint32_t k = 0; k < K; ++k) {
      const double f = fbl[k * bd + tid];
      const double *e = ebl + k * 16;
#pragma unroll
      for (int r = 0; r < 16; ++r) lam[r] = fma(f, e[r], lam[r]);
    }
#pragma unroll
    for (int r = 15; r >= 0; --r) {
      const uint32_t t = tb + r;
      real out = (real)0;
      if (t >= 1 && t <= T) {
        double L = lam[r];
        if ((int64_t)t <= u_reg) L += creg;
        if (PLUS && ema) {
          while (sp_i >= 0 && st[sp_i] > t) {
            --sp_i;
            f_sp = sp_i >= 0 ? (double)phi_row[st[sp_i]] : 0.0;
          }
          const double f = sp_i >= 0 ? f_sp * pow(n.beta_f, (double)(t - st[sp_i])) : 0.0;
          R = ((int64_t)t <= u_reg ? n.c_reg * (1.0 - n.beta_f) * (f - n.f_target) : 0.0) + n.beta_f * R;
          L += R;
        }
        const double p = (double)ps[r];
        const double pl = p * L;
        // with the full reset the membrane's derivative restarts after a
        // spike of this neuron at step t: alpha (1 - z^t)
        const bool zt = PLUS && n.reset_mode == 1 && inrow && ((zrow[(size_t)t * n.Jw] >> (j & 63u)) & 1ull);
        const double m0 = pl + (zt ? 0.0 : n.alpha_d) * mu0 + p * mu1;
        const double m1 = -beta * pl + (n.rho_d - p * beta) * mu1;
        mu0 = m0;
        mu1 = m1;
        out = (real)m0;
      }
      tile[tid * 17 + r] = out;
    }
    __syncthreads();
    // each store: 4 rows x 16 consecutive steps of this wavefront's 64 rows
#pragma unroll 4
    for (uint32_t it = 0; it < 16; ++it) {
      const uint32_t row = it * 4 + (lane >> 4), r = lane & 15u;
      const uint32_t jj = blockIdx.x * bd + wbase + row, t = tb + r;
      if (jj < n.J && t >= 1 && t <= T) n.phi[((size_t)b * n.Jp + jj) * n.Tp + t] = tile[(wbase + row) * 17 + r];
    }
  }
  if (!live) return;
  real *go = n.gout_b + (size_t)b * K * n.Jp + j;
  const double *eo = n.ebo + (size_t)b * (n.Tcap + 2) * K;
  for (uint32_t k = 0; k < K; ++k) {
    double acc = 0.0;
    for (uint32_t i = 0; i < c; ++i) acc += eo[(size_t)st[i] * K + k];
    go[(size_t)k * n.Jp] = (real)acc;
  }
}

// Per-source spike table of the batch.  The synapse kernel visits the
// synapses of a target, whose sources are scattered; keeping all of a
// source's spike times of a trial chunk in one contiguous record lets a
// lane fetch them with one line read instead of two per trial.  A record
// of u 16-byte units takes 1, 2 or 4 units (u up to 4) or a multiple of 8
// (u above 4), in a region of the table for its size class, each region
// starting on a 128-byte line, so that no record crosses a line (a read of
// a record costs the lines it touches).  Within a class, records are
// chunk-major and source-minor; their offsets come from a three-kernel
// exclusive scan of the rounded sizes, one per class.
__device__ inline uint32_t pk_class(uint32_t u) { return u > 4u ? 0u : u > 2u ? 1u : u > 1u ? 2u : 3u; }
__device__ inline uint32_t pk_rounded(uint32_t u) { return u > 4u ? (u + 7u) & ~7u : u > 2u ? 4u : u; }

template <typename real>
__device__ inline uint32_t pk_units(const DevNet<real> &n, uint32_t e, uint32_t ginst, uint32_t ntr) {
  const uint32_t c = e / n.NS, i = e - c * n.NS;
  const uint32_t b0 = c * ginst;
  if (b0 >= ntr) return 0;
  const uint32_t nb = min(ginst, ntr - b0);
  uint32_t tot = 0;
  for (uint32_t bi = 0; bi < nb; ++bi) tot += n.spk_cnt[(size_t)(b0 + bi) * n.NS + i];
  return tot ? 1u + (tot + 7u) / 8u : 0u;
}

// Block-local exclusive scans of the rounded record sizes, per size class
// (kScanItems records per block): the record's place within its class and
// block into pk_off, the block's class totals into pk_bsum[block][class].
template <typename real>
__global__ __launch_bounds__(1024) void k_pack_scan_local(DevNet<real> n, uint32_t ginst, uint32_t N) {
  __shared__ uint32_t wsum[17];
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const uint32_t e0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t sz[4];
#pragma unroll
  for (uint32_t u = 0; u < 4; ++u) sz[u] = e0 + u < N ? pk_units(n, e0 + u, ginst, ntr) : 0u;
  uint32_t off[4] = {kNoRecord, kNoRecord, kNoRecord, kNoRecord};
  for (uint32_t c = 0; c < 4; ++c) {
    uint32_t tsum = 0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) tsum += sz[u] && pk_class(sz[u]) == c ? pk_rounded(sz[u]) : 0u;
    uint32_t tot;
    uint32_t run = block_exclusive_scan(tsum, wsum, &tot);
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u)
      if (sz[u] && pk_class(sz[u]) == c) {
        off[u] = run;
        run += pk_rounded(sz[u]);
      }
    if (threadIdx.x == 0) n.pk_bsum[(size_t)blockIdx.x * 4 + c] = tot;
    __syncthreads();  // (wsum is reused by the next class)
  }
#pragma unroll
  for (uint32_t u = 0; u < 4; ++u)
    if (e0 + u < N) n.pk_off[e0 + u] = off[u];
}

// Exclusive scans of the block totals per class (one block), and the start
// of each class's region: pk_bsum[nblk][class], classes in order 0..3 (the
// longest records first), each region on a 128-byte line.
template <typename real>
__global__ __launch_bounds__(1024) void k_pack_scan_blocks(DevNet<real> n, uint32_t nblk) {
  __shared__ uint32_t wsum[17];
  uint32_t start = 0;
  for (uint32_t c = 0; c < 4; ++c) {
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nblk; base += blockDim.x) {
      const uint32_t i = base + threadIdx.x;
      const uint32_t x = i < nblk ? n.pk_bsum[(size_t)i * 4 + c] : 0u;
      uint32_t tot;
      const uint32_t pre = block_exclusive_scan(x, wsum, &tot);
      __syncthreads();
      if (i < nblk) n.pk_bsum[(size_t)i * 4 + c] = carry + pre;
      carry += tot;
    }
    if (threadIdx.x == 0) n.pk_bsum[(size_t)nblk * 4 + c] = start;
    start = (start + carry + 7u) & ~7u;
  }
}

// Final offsets, headers (counts of the chunk's trials) and the LDS indices
// of the spikes.  Also counts, per source, the deliveries that arrive within
// their trial and the (synapse, trial) pairs with at least one, from the
// source's out-degree per delay.
template <typename real>
__global__ __launch_bounds__(256) void k_pack_fill(DevNet<real> n, uint32_t ginst, uint32_t N, uint32_t nblk) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long nev = 0, nfl = 0;
  if (e < N && n.pk_off[e] != kNoRecord) {
    const uint32_t ntr = n.ctl[CTL_NTRIALS];
    const uint32_t cls = pk_class(pk_units(n, e, ginst, ntr));
    const uint32_t off = n.pk_off[e] + n.pk_bsum[(size_t)(e / kScanItems) * 4 + cls] + n.pk_bsum[(size_t)nblk * 4 + cls];
    n.pk_off[e] = off;
    const uint32_t c = e / n.NS, i = e - c * n.NS;
    const uint32_t b0 = c * ginst, nb = min(ginst, ntr - b0);
    const uint32_t *od = n.outdeg + (size_t)i * n.R;
    uint32_t h[4] = {0, 0, 0, 0};
    uint16_t *dst = n.pk + (size_t)off * 8 + 8;
    uint32_t tot = 0;
    for (uint32_t bi = 0; bi < nb; ++bi) {
      const uint32_t b = b0 + bi, T = n.T[b];
      const uint32_t cnt = n.spk_cnt[(size_t)b * n.NS + i];
      h[bi >> 1] |= cnt << ((bi & 1u) * 16u);
      const uint16_t *src = n.spk_t + (size_t)b * n.spk_stride + (size_t)i * n.Lc;
      for (uint32_t k = 0; k < cnt; ++k) dst[tot + k] = (uint16_t)(bi * n.Ts + src[k]);
      tot += cnt;
      if (cnt == 0) continue;
      for (uint32_t d = 1; d < n.R; ++d) {
        const uint32_t deg = od[d];
        if (deg == 0 || src[0] + d > T) continue;
        uint32_t m = cnt;  // spikes arriving by step T (times ascending)
        while (m > 0 && src[m - 1] + d > T) --m;
        nev += (unsigned long long)deg * m;
        nfl += deg;
      }
    }
    const uint16_t zero_slot = (uint16_t)(ginst * n.Ts);
    for (uint32_t k = tot; k < (tot + 7u) / 8u * 8u; ++k) dst[k] = zero_slot;
    reinterpret_cast<uint4 *>(n.pk)[off] = make_uint4(h[0], h[1], h[2], h[3]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    nev += __shfl_down(nev, o);
    nfl += __shfl_down(nfl, o);
  }
  if ((threadIdx.x & 63u) == 0) {
    if (nev) atomicAdd(&n.evcnt[(blockIdx.x * 4 + (threadIdx.x >> 6)) & 63u], nev);
    if (nfl) atomicAdd(&n.cnt[CNT_FLUSH], nfl);
  }
}

// Event-driven synapse gradient, target-major.  Block (j, c) handles the
// incoming synapses of target j for the trials of chunk c (at most 8).  The
// target's archive rows phi[b][j][.] of those trials are staged in LDS, one
// row of Ts entries per trial that holds phi^t for t = 1..T_b and zeros
// after it (and a zero tail after the last row), so that an arrival
// a = s + D beyond its trial reads a zero.  Each lane takes a synapse, reads
// its source's record of the spike table (the header and the first blocks
// of LDS indices issued together) and adds phl[index + D] for every element
// (Kahan); padding elements index the zero tail.  With one chunk the sum
// goes straight into the accumulator pair (gs, gc); otherwise into
// partial[c][q] for a fixed-order reduction.
// PRE: blocks of 8 spike indices loaded together with a record's header (a
// shape choice: records of sparse sources hold one or two blocks)

template <typename real>
__device__ inline void add_block(uint4 v, const real *base, real &s, real &c) {
  const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (uint32_t e = 0; e < 8; ++e) kahan_add(s, c, base[(w4[e >> 1] >> ((e & 1u) * 16u)) & 0xFFFFu]);
}

// Synapse-kernel variants: spike-index blocks loaded with a record's header
// (PRE) and synapses a thread takes at a time (B), whose loads are all
// issued before any of their gradient stores (vector memory operations
// complete in order, so a load issued after a store waits for it).
constexpr uint32_t kSynVariants = 7;
__host__ __device__ constexpr uint32_t syn_pre_of(uint32_t v) { return v == 0 ? 5u : v == 2 || v == 4 ? 2u : 1u; }
__host__ __device__ constexpr uint32_t syn_batch_of(uint32_t v) {
  return v == 6 ? 8u : v == 3 ? 4u : v == 4 || v == 5 ? 2u : 1u;
}

template <typename real, uint32_t PRE, uint32_t B>
__global__ __launch_bounds__(256) void k_synapse(DevNet<real> n, uint32_t ginst, uint32_t nchunk, real *partial) {
  constexpr uint32_t GB = 8;
  extern __shared__ __align__(16) unsigned char syn_smem[];
  real *phl = reinterpret_cast<real *>(syn_smem);   // [ginst][Ts] + zero tail [R]
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const uint32_t c = blockIdx.x % nchunk, j = blockIdx.x / nchunk;
  const uint32_t b0 = c * ginst, nb = min(min(ginst, ntr - b0), GB);
  const uint32_t tid = threadIdx.x;
  for (uint32_t bi = 0; bi < nb; ++bi) {
    const real *src = n.phi + ((size_t)(b0 + bi) * n.Jp + j) * n.Tp;
    real *dst = phl + bi * n.Ts;
    const uint32_t T = n.T[b0 + bi];
    for (uint32_t t = tid; t < n.Ts; t += 4 * blockDim.x) {
      real v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t tt = t + u * blockDim.x;
        v[u] = (tt >= 1 && tt <= T) ? src[tt] : (real)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t + u * blockDim.x < n.Ts) dst[t + u * blockDim.x] = v[u];
    }
  }
  for (uint32_t t = tid; t < n.R; t += blockDim.x) phl[ginst * n.Ts + t] = (real)0;
  __syncthreads();
  const uint4 *pk4 = reinterpret_cast<const uint4 *>(n.pk);
  const uint32_t *poff = n.pk_off + (size_t)c * n.NS;
  const uint32_t q1 = n.tm_ptr[j + 1];
  for (uint32_t q0 = n.tm_ptr[j] + tid; q0 < q1; q0 += B * blockDim.x) {
    // loads of the thread's B synapses, level by level, from valid addresses
    // (a synapse beyond the row reads synapse q0; a source without a record
    // reads record 0: the table has slack beyond its last record, so every
    // header load stays in bounds)
    uint32_t pkv[B], ov[B];
#pragma unroll
    for (uint32_t u = 0; u < B; ++u) {
      const uint32_t q = q0 + u * blockDim.x;
      pkv[u] = n.tm_syn[q < q1 ? q : q0];
    }
#pragma unroll
    for (uint32_t u = 0; u < B; ++u) ov[u] = q0 + u * blockDim.x < q1 ? poff[pkv[u] & 0xFFFFFFu] : kNoRecord;
    uint4 pre[B][PRE + 1];
#pragma unroll
    for (uint32_t u = 0; u < B; ++u) {
      const uint4 *rec = pk4 + (ov[u] != kNoRecord ? ov[u] : 0u);
#pragma unroll
      for (uint32_t v = 0; v <= PRE; ++v) pre[u][v] = rec[v];
    }
    real gsv[B], gcv[B];
    if (nchunk == 1) {
#pragma unroll
      for (uint32_t u = 0; u < B; ++u) {
        const uint32_t q = q0 + u * blockDim.x, qs = q < q1 ? q : q0;
        gsv[u] = n.g_fresh ? (real)0 : n.gs[qs];
        gcv[u] = n.g_fresh ? (real)0 : n.gc[qs];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < B; ++u) {
      const uint32_t q = q0 + u * blockDim.x;
      if (q >= q1) break;
      real s = 0, cc = 0;
      if (ov[u] != kNoRecord) {
        const uint4 h = pre[u][0];
        const uint32_t total = (h.x & 0xFFFFu) + (h.x >> 16) + (h.y & 0xFFFFu) + (h.y >> 16) + (h.z & 0xFFFFu) +
                               (h.z >> 16) + (h.w & 0xFFFFu) + (h.w >> 16);
        const uint32_t nbk = (total + 7u) >> 3;
        const real *base = phl + (pkv[u] >> 24);
#pragma unroll
        for (uint32_t v = 0; v < PRE; ++v)
          if (v < nbk) add_block(pre[u][v + 1], base, s, cc);
        for (uint32_t v = PRE; v < nbk; ++v) add_block(pk4[ov[u] + v + 1], base, s, cc);
      }
      if (nchunk == 1) {
        kahan_add(gsv[u], gcv[u], s);
        kahan_add(gsv[u], gcv[u], cc);
        n.gs[q] = gsv[u];
        n.gc[q] = gcv[u];
      } else {
        partial[(size_t)c * n.S + q] = s + cc;
      }
    }
  }
}

// ---------------------------------------------------- time-driven baseline
// The gradient of Alg. 1 ("time-driven gradient computation"), evaluated
// the way a time-driven simulator does it: every synapse, every step.  Kept
// as the baseline the event-driven path is measured against; same inputs
// (spike bitsets, psi archive, error signal) and the same accumulators.

// L_j^t = sum_k B_jk E_k^t (eq. final-gradient), FP64 sum, stored per
// (trial, step, neuron) at the step u = t - d whose eligibility it meets
// (readout delay d), and only for t <= T - d^ls (learning-signal delay).
template <typename real>
__global__ __launch_bounds__(256) void k_learning_signal(DevNet<real> n, real *L) {
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const uint64_t per = (uint64_t)n.Jp * n.Tp;  // neuron-major: L[b][j][u], u < Tp
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)ntr * per;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t b = (uint32_t)(i / per);
    const uint32_t j = (uint32_t)((i % per) / n.Tp), u = (uint32_t)(i % n.Tp);
    const uint64_t t = (uint64_t)u + n.d_out;
    double acc = 0.0;
    if (j < n.J && u >= 1 && u <= n.Tcap && t + n.d_ls <= n.T[b]) {
      const double *E = n.err + ((size_t)b * (n.Tcap + 2) + t) * n.K;
      for (uint32_t k = 0; k < n.K; ++k) acc += (double)n.fb[(size_t)j * n.K + k] * E[k];
    }
    L[i] = (real)acc;
  }
}

// psi[b][t][j] (time-major, as the forward pass writes it) -> out[b][j][t]
// (neuron-major, row length Tp), through 64 x 64 LDS tiles.
template <typename real>
__global__ __launch_bounds__(256) void k_transpose_psi(DevNet<real> n, real *out) {
  __shared__ real tile[64][65];
  const uint32_t b = blockIdx.z;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t t0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const uint32_t tx = threadIdx.x & 63u, ty = threadIdx.x >> 6;  // 4 rows per pass
  for (uint32_t r = ty; r < 64; r += 4) {
    const uint32_t t = t0 + r, j = j0 + tx;
    tile[r][tx] = t <= n.Tcap && j < n.Jp ? n.psi[((size_t)b * (n.Tcap + 1) + t) * n.Jp + j] : (real)0;
  }
  __syncthreads();
  for (uint32_t r = ty; r < 64; r += 4) {
    const uint32_t j = j0 + r, t = t0 + tx;
    if (j < n.Jp && t < n.Tp) out[((size_t)b * n.Jp + j) * n.Tp + t] = tile[tx][r];
  }
}

// The time-driven gradient with one workgroup per (target j, trial chunk
// c): the target's psi and learning-signal rows of the chunk's trials are
// staged in LDS once (neuron-major copies), and each thread runs the
// eligibility recursion of eq. eligibility-vector-substituted and eq.
// filtered-eligibility-trace for one incoming synapse at a time over every
// step of every trial of the chunk, with e, ebar in registers; the arrival
// indicator x^t comes from the source's spike-time list (emission steps,
// ascending) and the full reset from the target's own.  Sums, counts and
// the regulariser term as in k_td_synapse.  LDS: 2 * ginst * Tp reals.
template <typename real>
__global__ __launch_bounds__(256) void k_td_target(DevNet<real> n, const real *L, const real *psnm, uint32_t ginst,
                                                   uint32_t nchunk, real *partial) {
  extern __shared__ __align__(16) unsigned char td_smem[];
  real *lps = reinterpret_cast<real *>(td_smem);  // [ginst][Tp] psi rows
  real *lL = lps + (size_t)ginst * n.Tp;          // [ginst][Tp] learning-signal rows
  const uint32_t j = blockIdx.x, c = blockIdx.y;
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const uint32_t b0 = c * ginst, nb = b0 < ntr ? min(ginst, ntr - b0) : 0u;
  if (j >= n.J || nb == 0) return;
  for (uint32_t bi = 0; bi < nb; ++bi) {
    const size_t row = ((size_t)(b0 + bi) * n.Jp + j) * n.Tp;
    for (uint32_t t = threadIdx.x; t < n.Tp; t += blockDim.x) {
      lps[(size_t)bi * n.Tp + t] = psnm[row + t];
      lL[(size_t)bi * n.Tp + t] = L[row + t];
    }
  }
  __syncthreads();
  const real beta = n.beta_j[j];
  const real kappa = (real)n.kappa_e_d;
  unsigned long long nev = 0, nfl = 0;
  const uint32_t q1 = n.tm_ptr[j + 1];
  for (uint32_t q = n.tm_ptr[j] + threadIdx.x; q < q1; q += blockDim.x) {
    const uint32_t pk = n.tm_syn[q];
    const uint32_t src = pk & 0xFFFFFFu, D = pk >> 24;
    real s = 0, cc = 0;
    for (uint32_t bi = 0; bi < nb; ++bi) {
      const uint32_t b = b0 + bi, T = n.T[b];
      const real *ps = lps + (size_t)bi * n.Tp, *Lb = lL + (size_t)bi * n.Tp;
      // arrivals: the source's emission steps + D, in order
      const uint16_t *st = n.spk_t + (size_t)b * n.spk_stride + (size_t)src * n.Lc;
      const uint32_t cnt = n.spk_cnt[(size_t)b * n.NS + src];
      uint32_t ci = 0, next = cnt ? (uint32_t)st[0] + D : 0xFFFFFFFFu;
      // the target's own spikes (full reset: the membrane component restarts after them)
      const uint16_t *sj = n.spk_t + (size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Lc;
      const uint32_t cj = n.reset_mode == 1 ? n.spk_cnt[(size_t)b * n.NS + n.I + j] : 0u;
      uint32_t ri = 0, rnext = cj ? (uint32_t)sj[0] + 1u : 0xFFFFFFFFu;
      real ev = 0, ea = 0, eb = 0, psi_prev = 0, es = 0, ec = 0;
      const uint32_t t_reg = T > n.d_out ? T - n.d_out : 0u;
      uint32_t arrivals = 0;
      for (uint32_t t = 1; t <= T; ++t) {
        const bool x = t == next;
        if (x) {
          ++ci;
          next = ci < cnt ? (uint32_t)st[ci] + D : 0xFFFFFFFFu;
        }
        const bool zr = t == rnext;
        if (zr) {
          ++ri;
          rnext = ri < cj ? (uint32_t)sj[ri] + 1u : 0xFFFFFFFFu;
        }
        arrivals += x ? 1u : 0u;
        const real psi_now = ps[t];
        const real ea_new = psi_prev * ev + (n.rho - psi_prev * beta) * ea;
        const real ev_new = (zr ? (real)0 : n.alpha) * ev + (x ? (real)1 : (real)0);
        const real e = psi_now * (ev_new - beta * ea_new);
        eb = kappa * eb + e;
        ev = ev_new;
        ea = ea_new;
        psi_prev = psi_now;
        kahan_add(s, cc, Lb[t] * eb);
        if (t <= t_reg) kahan_add(es, ec, e);
      }
      if (n.c_reg != 0.0) {
        const double creg = n.c_reg / (double)T *
                            ((double)n.spk_cnt[(size_t)b * n.NS + n.I + j] / (double)T - n.f_target);
        kahan_add(s, cc, (real)(creg * ((double)es + (double)ec)));
      }
      nev += arrivals;
      nfl += arrivals ? 1u : 0u;
    }
    if (nchunk == 1) {
      real gs = n.g_fresh ? (real)0 : n.gs[q], gc = n.g_fresh ? (real)0 : n.gc[q];
      kahan_add(gs, gc, s);
      kahan_add(gs, gc, cc);
      n.gs[q] = gs;
      n.gc[q] = gc;
    } else {
      partial[(size_t)c * n.S + q] = s + cc;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    nev += __shfl_down(nev, o);
    nfl += __shfl_down(nfl, o);
  }
  if ((threadIdx.x & 63u) == 0) {
    if (nev) atomicAdd(&n.evcnt[((blockIdx.x + blockIdx.y) * 4 + (threadIdx.x >> 6)) & 63u], nev);
    if (nfl) atomicAdd(&n.cnt[CNT_FLUSH], nfl);
  }
}

// One thread per (synapse q, trial chunk c): the eligibility recursion of
// eq. eligibility-vector-substituted and eq. filtered-eligibility-trace over
// every step of each trial of the chunk, g += L^{t+d} ebar^t (Kahan; L as
// stored by k_learning_signal), plus the rate regulariser c^reg/T (f_j - f*)
// times the sum of e^t over t <= T - d.  The arrival indicator x^t is the
// source's spike bit at step t - D.
template <typename real>
__global__ __launch_bounds__(256) void k_td_synapse(DevNet<real> n, const real *L, uint32_t ginst, uint32_t nchunk,
                                                    real *partial) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long nev = 0, nfl = 0;
  if (gid < n.S * nchunk) {
    const uint32_t c = (uint32_t)(gid / n.S);
    const uint64_t q = gid - (uint64_t)c * n.S;
    uint32_t lo = 0, hi = n.J;  // target of q: tm_ptr[lo] <= q < tm_ptr[lo + 1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (n.tm_ptr[mid] <= q) lo = mid; else hi = mid;
    }
    const uint32_t j = lo;
    const uint32_t pk = n.tm_syn[q];
    const uint32_t src = pk & 0xFFFFFFu, D = pk >> 24;
    const bool is_in = src < n.I;
    const uint32_t si = is_in ? src : src - n.I;
    const real beta = n.beta_j[j];
    const real kappa = (real)n.kappa_e_d;  // the eligibility trace's filter
    const uint32_t ntr = n.ctl[CTL_NTRIALS];
    const uint32_t b0 = c * ginst, nb = b0 < ntr ? min(ginst, ntr - b0) : 0u;
    real s = 0, cc = 0;
    for (uint32_t bi = 0; bi < nb; ++bi) {
      const uint32_t b = b0 + bi, T = n.T[b];
      const real *ps = n.psi + (size_t)b * (n.Tcap + 1) * n.Jp + j;
      const real *Lb = L + ((size_t)b * n.Jp + j) * n.Tp;
      real ev = 0, ea = 0, eb = 0, psi_prev = 0, es = 0, ec = 0;
      const uint32_t t_reg = T > n.d_out ? T - n.d_out : 0u;
      uint32_t arrivals = 0;
      for (uint32_t t = 1; t <= T; ++t) {
        uint32_t x = 0;
        if (t >= D) {
          const uint32_t se = t - D;  // emission step
          if (is_in) {
            x = (uint32_t)(n.in_bits[((size_t)b * n.Tcap + se) * n.Iw + (si >> 6)] >> (si & 63u)) & 1u;
          } else if (se >= 1) {
            x = (uint32_t)(n.rec_bits[((size_t)b * (n.Tcap + 1) + se) * n.Jw + (si >> 6)] >> (si & 63u)) & 1u;
          }
        }
        arrivals += x;
        const real psi_now = ps[(size_t)t * n.Jp];
        const real ea_new = psi_prev * ev + (n.rho - psi_prev * beta) * ea;
        // full reset: the membrane component restarts after a spike of j at t - 1
        const bool zr = n.reset_mode == 1 &&
                        ((n.rec_bits[((size_t)b * (n.Tcap + 1) + t - 1) * n.Jw + (j >> 6)] >> (j & 63u)) & 1ull);
        const real ev_new = (zr ? (real)0 : n.alpha) * ev + (real)x;
        const real e = psi_now * (ev_new - beta * ea_new);
        eb = kappa * eb + e;
        ev = ev_new;
        ea = ea_new;
        psi_prev = psi_now;
        kahan_add(s, cc, Lb[t] * eb);
        if (t <= t_reg) kahan_add(es, ec, e);
      }
      if (n.c_reg != 0.0) {
        const double creg = n.c_reg / (double)T *
                            ((double)n.spk_cnt[(size_t)b * n.NS + n.I + j] / (double)T - n.f_target);
        kahan_add(s, cc, (real)(creg * ((double)es + (double)ec)));
      }
      nev += arrivals;
      nfl += arrivals ? 1u : 0u;
    }
    if (nchunk == 1) {
      real gs = n.g_fresh ? (real)0 : n.gs[q], gc = n.g_fresh ? (real)0 : n.gc[q];
      kahan_add(gs, gc, s);
      kahan_add(gs, gc, cc);
      n.gs[q] = gs;
      n.gc[q] = gc;
    } else {
      partial[(size_t)c * n.S + q] = s + cc;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    nev += __shfl_down(nev, o);
    nfl += __shfl_down(nfl, o);
  }
  if ((threadIdx.x & 63u) == 0) {
    if (nev) atomicAdd(&n.evcnt[(blockIdx.x * 4 + (threadIdx.x >> 6)) & 63u], nev);
    if (nfl) atomicAdd(&n.cnt[CNT_FLUSH], nfl);
  }
}

// Output synapses, time-driven: zbar = F_kappa(z_j), g_kj += E_k^{t+d}
// zbar^t over t <= T - d (readout delay d), one thread per (trial, readout,
// neuron), FP64 sum.
template <typename real>
__global__ __launch_bounds__(256) void k_td_output(DevNet<real> n) {
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const uint64_t per = (uint64_t)n.K * n.Jp;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)ntr * per;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t b = (uint32_t)(i / per), k = (uint32_t)((i % per) / n.Jp), j = (uint32_t)(i % n.Jp);
    double zb = 0.0, g = 0.0;
    if (j < n.J) {
      const uint32_t T = n.T[b], d = n.d_out;
      for (uint32_t t = 1; t + d <= T; ++t) {
        const uint32_t z = (uint32_t)(n.rec_bits[((size_t)b * (n.Tcap + 1) + t) * n.Jw + (j >> 6)] >> (j & 63u)) & 1u;
        zb = n.kappa_d * zb + (double)z;
        g += n.err[((size_t)b * (n.Tcap + 2) + t + d) * n.K + k] * zb;
      }
    }
    n.gout_b[i] = (real)g;
  }
}

// ------------------------------------------------- e-prop+ update schedule
// One network instance runs its samples back to back (Results, "Continuous
// dynamics").  Every presynaptic spike first updates its synapse's weight by
// gradient descent over the eligibility steps whose learning signal has
// reached the neuron (Results, "Weight updates with every spike"; Alg.
// "event-driven weight update" evaluated at each spike), then is delivered
// with the new weight.  A thread per target neuron walks its incoming
// synapses in target-major order, so the input current sums in the canonical
// order and each weight has a single writer; weights live in tm_w for the
// run and are copied to the delivery table afterwards (scatter delivery).

template <typename real>
__global__ __launch_bounds__(256) void k_online_fill(DevNet<real> n, int to_records) {
  if (!n.dlw) return;  // gather delivery: tm_w is the only copy of the weights
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n.S; q += (uint64_t)gridDim.x * blockDim.x) {
    real *wp = reinterpret_cast<real *>(n.dlw + n.tm_dpos[q]);
    if (to_records) *wp = n.tm_w[q];
    else n.tm_w[q] = *wp;
  }
}

// Did source src (input or recurrent) emit a spike at step s of the run?
template <typename real>
__device__ inline bool online_spiked(const DevNet<real> &n, uint32_t src, int64_t s) {
  if (src < n.I) return s >= 0 && s < (int64_t)n.Tcap && ((n.in_bits[(size_t)s * n.Iw + (src >> 6)] >> (src & 63u)) & 1ull);
  const uint32_t r = src - n.I;
  return s >= 1 && ((n.rec_bits[(size_t)s * n.Jw + (r >> 6)] >> (r & 63u)) & 1ull);
}

// The update walk of one synapse (i -> j, delay D) at an arrival at step t:
// its eligibility steps s_done+1 .. t - lag (eq. eligibility-vector-
// substituted, eq. filtered-eligibility-trace, the cutoff rule), each adding
// L_j^{s+d} ebar^s (the run's learning-signal history) and the
// moving-average regulariser's c (f_j^s - f*) G_beta(e^s);
// returns the new weight w - eta g and stores it and the trace state.
template <typename real>
__device__ inline real online_update(const DevNet<real> &n, const OnlineRun<real> &o, uint32_t j, uint32_t q,
                                     uint32_t t, real beta, bool ema) {
  const uint32_t pk = n.tm_syn[q];
  const uint32_t src = pk & 0xFFFFFFu, D = pk >> 24;
  OnlineSyn<real> st = o.syn[q];
  const int64_t s_new = (int64_t)t - o.lag;
  double g = 0.0;
  real pp = n.psi[(size_t)st.s_done * n.Jp + j];  // psi of the step before the next one
  for (int64_t s = (int64_t)st.s_done + 1; s <= s_new; ++s) {
    const bool x = online_spiked(n, src, s - D);
    const real pn = n.psi[(size_t)s * n.Jp + j];
    if (x) st.last = (uint32_t)s;
    if (o.cutoff && (st.last == 0 || (uint64_t)(s - st.last) >= o.cutoff)) {
      // beyond eprop_isi_trace_cutoff the traces count as decayed
      st.ev = st.ea = st.eb = st.gh = (real)0;
      pp = pn;
      continue;
    }
    const bool zr = n.reset_mode == 1 && ((n.rec_bits[(size_t)(s - 1) * n.Jw + (j >> 6)] >> (j & 63u)) & 1ull);
    const real ea_new = pp * st.ev + (n.rho - pp * beta) * st.ea;
    const real ev_new = (zr ? (real)0 : n.alpha) * st.ev + (x ? (real)1 : (real)0);
    const real e = pn * (ev_new - beta * ea_new);
    st.eb = (real)n.kappa_e_d * st.eb + e;
    st.ev = ev_new;
    st.ea = ea_new;
    st.gh = (real)n.beta_f * st.gh + ((real)1 - (real)n.beta_f) * e;
    g += (double)o.Lh[(size_t)(s + n.d_out) * n.Jp + j] * (double)st.eb;
    if (ema) g += n.c_reg * ((double)o.fh[(size_t)s * n.Jp + j] - n.f_target) * (double)st.gh;
    pp = pn;
  }
  if (s_new > (int64_t)st.s_done) st.s_done = (uint32_t)s_new;
  o.syn[q] = st;
  const real w = (real)((double)n.tm_w[q] - o.eta * g);
  n.tm_w[q] = w;
  return w;
}

// The synapse side of step t: a wavefront per target neuron scans its
// incoming synapses in target-major order, gathers the ones with an arrival
// into a list held one per lane (in that order), lets the lanes run their
// update walks side by side whenever the list is full or the scan ends, and
// adds the new weights to the input current in list order, so the sum keeps
// the canonical order.  The current goes to Ibuf for the neuron update.
template <typename real>
__global__ __launch_bounds__(256) void k_online_syn(DevNet<real> n, OnlineRun<real> o, uint32_t t) {
  const uint32_t lane = lane_id();
  const uint32_t j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n.J) return;  // whole wavefronts
  const real beta = n.beta_j[j];
  const bool ema = n.reg_mode == 1;
  real I = 0;            // the same in every lane
  uint32_t cnt = 0;      // arrivals in the list (the same in every lane)
  uint32_t pend = 0;     // this lane's list entry (lanes < cnt)
  unsigned long long nev = 0;
  const uint32_t q0 = n.tm_ptr[j], q1 = n.tm_ptr[j + 1];
  auto run_list = [&]() {
    real w = (real)0;
    if (lane < cnt) w = online_update(n, o, j, pend, t, beta, ema);
    for (uint32_t l = 0; l < cnt; ++l) I = I + __shfl(w, (int)l);
    nev += cnt;
    cnt = 0;
  };
  for (uint32_t qb = q0; qb < q1; qb += 64) {
    const uint32_t q = qb + lane;
    bool hit = false;
    if (q < q1) {
      const uint32_t pk = n.tm_syn[q];
      hit = online_spiked(n, pk & 0xFFFFFFu, (int64_t)t - (pk >> 24));
    }
    const uint64_t m = __ballot(hit);
    const uint32_t nh = (uint32_t)__popcll(m);
    if (nh == 0) continue;
    if (cnt + nh > 64) run_list();
    // slot cnt + r takes the r-th arrival of this chunk
    const bool mine = lane >= cnt && lane < cnt + nh;
    const uint32_t from = mine ? nth_set_bit(m, lane - cnt) : lane;
    const uint32_t qv = (uint32_t)__shfl((int)q, (int)from);
    if (mine) pend = qv;
    cnt += nh;
  }
  if (cnt) run_list();
  if (lane == 0) {
    o.Ibuf[j] = I;
    if (nev) atomicAdd(&n.evcnt[(blockIdx.x * 4 + (threadIdx.x >> 6)) & 63u], nev);
  }
}

// The neuron side of step t (a thread per neuron): the update with the
// current gathered by k_online_syn, spikes, rates.
template <typename real, bool FORCED>
__global__ __launch_bounds__(256) void k_online_neuron(DevNet<real> n, OnlineRun<real> o, uint32_t t) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n.Jp) return;  // whole wavefronts: Jp is a multiple of 64
  const bool live = j < n.J;
  const bool ema = n.reg_mode == 1;
  const real I = live ? o.Ibuf[j] : (real)0;
  real v = n.v[j], a = n.a[j];
  uint8_t stt = n.nst[j];
  const bool z = neuron_step<real, FORCED>(n, 0, t, j, live, I, n.beta_j[j], v, a, stt);
  n.v[j] = v;
  n.a[j] = a;
  n.nst[j] = stt;
  const uint64_t word = publish_bits(n, 0, t, j, z);
  if (ema)
    o.fh[(size_t)t * n.Jp + j] =
        (real)n.beta_f * o.fh[(size_t)(t - 1) * n.Jp + j] + ((real)1 - (real)n.beta_f) * (z ? (real)1 : (real)0);
  if (lane_id() == 0 && word) atomicAdd(&n.cnt[CNT_REC_SPIKES], (unsigned long long)__popcll(word));
}

// L_j^t = sum_k B_jk E_k^t (eq. final-gradient) of every neuron, FP64 sum in
// ascending k, kept for the walks of later steps.
template <typename real>
__global__ __launch_bounds__(256) void k_online_learn(DevNet<real> n, OnlineRun<real> o, uint32_t t) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n.J) return;
  const double *E = o.Eh + (size_t)t * n.K;
  double L = 0.0;
  for (uint32_t k = 0; k < n.K; ++k) L = L + (double)n.fb[(size_t)j * n.K + k] * E[k];
  o.Lh[(size_t)t * n.Jp + j] = (real)L;
}

// One block: the readout synapses of neurons whose spike of step t - d
// reaches the readout now (gradient E_k^{r+d} zbar_j^r over the steps not
// yet used, eq. eprop-output-new-subs-rewritten), then the readout
// (eq. leaky_integrator_with_delay), error signal and loss of step t, FP64.
// Readout synapses of the neurons whose spike reaches the readout at step t
// (emitted at t - d): each walks its readout traces over the steps not yet
// used, r <= t - 1 - d, and takes one gradient-descent step with
// E^{r+d} zbar^r.  One thread per (spike-bitset word, output k), a block
// holding whole words, so a neuron's walks for all outputs run side by side;
// after a barrier (every walk has read the neuron's old trace state), one
// thread per word walks once more without the error terms and stores the
// neuron's new state (zbar, last spike, last step used).
template <typename real>
__device__ inline void online_out_walk(const DevNet<real> &n, const OnlineRun<real> &o, uint32_t j, int64_t r0,
                                       int64_t r1, uint32_t &zl, double &zb, uint32_t k, double *g) {
  const uint32_t K = n.K, d = n.d_out;
  for (int64_t r = r0; r <= r1; ++r) {
    const bool x = (n.rec_bits[(size_t)r * n.Jw + (j >> 6)] >> (j & 63u)) & 1ull;
    if (x) zl = (uint32_t)r;
    if (o.cutoff && (zl == 0 || (uint64_t)(r - zl) >= o.cutoff)) {
      zb = 0.0;
      continue;
    }
    zb = n.kappa_d * zb + (x ? 1.0 : 0.0);
    if (g) *g += o.Eh[(size_t)(r + d) * K + k] * zb;
  }
}

template <typename real>
__global__ __launch_bounds__(256) void k_online_out_syn(DevNet<real> n, OnlineRun<real> o, uint32_t t) {
  const uint32_t K = n.K, d = n.d_out;
  if (t <= d) return;
  const uint32_t KB = min(K, blockDim.x), wpb = blockDim.x / KB;
  const uint32_t wl = threadIdx.x / KB, kk = threadIdx.x - wl * KB;
  const uint32_t w = blockIdx.x * wpb + wl;
  const bool on = wl < wpb && w < n.Jw;
  const uint64_t word0 = on ? n.rec_bits[(size_t)(t - d) * n.Jw + w] : 0ull;
  const int64_t r_new = (int64_t)t - 1 - d;
  for (uint64_t word = word0; word;) {
    const uint32_t j = w * 64 + (uint32_t)(__ffsll((unsigned long long)word) - 1);
    word &= word - 1ull;
    const uint32_t rd0 = o.r_done[j], zl0 = o.zlast[j];
    const double zb0 = o.zbo[j];
    for (uint32_t k = kk; k < K; k += KB) {
      uint32_t zl = zl0;
      double zb = zb0, g = 0.0;
      online_out_walk(n, o, j, (int64_t)rd0 + 1, r_new, zl, zb, k, &g);
      n.w_out[(size_t)k * n.Jp + j] = (real)((double)n.w_out[(size_t)k * n.Jp + j] - o.eta * g);
    }
  }
  __syncthreads();
  if (kk != 0) return;
  for (uint64_t word = word0; word;) {
    const uint32_t j = w * 64 + (uint32_t)(__ffsll((unsigned long long)word) - 1);
    word &= word - 1ull;
    const uint32_t rd0 = o.r_done[j];
    uint32_t zl = o.zlast[j];
    double zb = o.zbo[j];
    online_out_walk(n, o, j, (int64_t)rd0 + 1, r_new, zl, zb, 0u, (double *)nullptr);
    o.zbo[j] = zb;
    o.zlast[j] = zl;
    if (r_new > (int64_t)rd0) o.r_done[j] = (uint32_t)r_new;
  }
}

// Readout state, error signal and loss of step t (one block), after
// k_online_out_syn has updated the readout weights.
template <typename real>
__global__ __launch_bounds__(256) void k_online_readout(DevNet<real> n, OnlineRun<real> o, uint32_t t) {
  const uint32_t tid = threadIdx.x, K = n.K, d = n.d_out;
  __shared__ double red[256];
  __shared__ uint32_t smp;
  if (tid == 0) {
    uint32_t lo = 0, hi = o.n_samples;  // sample c with off[c] < t <= off[c + 1]
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (o.off[m] < t) lo = m; else hi = m;
    }
    smp = lo;
  }
  __syncthreads();
  const uint32_t c = smp;
  for (uint32_t k = tid; k < K; k += blockDim.x) {
    double sum = 0.0;
    if (t > d) {
      const uint64_t *row = n.rec_bits + (size_t)(t - d) * n.Jw;
      for (uint32_t w = 0; w < n.Jw; ++w) {
        uint64_t word = row[w];
        while (word) {
          const uint32_t j = w * 64 + (uint32_t)(__ffsll((unsigned long long)word) - 1);
          word &= word - 1ull;
          sum = sum + (double)n.w_out[(size_t)k * n.Jp + j];
        }
      }
    }
    o.y[k] = n.kappa_d * o.y[k] + sum;
  }
  __syncthreads();
  if (tid == 0) {
    const bool win = n.window ? n.window[t - 1] != 0 : true;
    const uint32_t label = n.loss != 0 ? o.label[c] : 0u;
    double *E = o.Eh + (size_t)t * K;
    double lp = 0.0;
    if (n.loss == 0) {
      for (uint32_t k = 0; k < K; ++k) {
        const double dd = o.y[k] - n.target[(size_t)(t - 1) * K + k];
        E[k] = win ? dd : 0.0;
        if (win) lp += 0.5 * dd * dd;
      }
    } else if (n.loss == 2) {
      for (uint32_t k = 0; k < K; ++k) {
        const double dd = o.y[k] - (k == label ? 1.0 : 0.0);
        E[k] = win ? 2.0 / K * dd : 0.0;
        if (win) {
          lp += dd * dd / K;
          o.psum[(size_t)c * K + k] += o.y[k];
        }
      }
    } else {
      double mx = o.y[0];
      for (uint32_t k = 1; k < K; ++k) mx = fmax(mx, o.y[k]);
      double se = 0.0;
      for (uint32_t k = 0; k < K; ++k) se += exp(o.y[k] - mx);
      for (uint32_t k = 0; k < K; ++k) {
        const double pi = exp(o.y[k] - mx) / se;
        E[k] = win ? pi - (k == label ? 1.0 : 0.0) : 0.0;
        if (win) o.psum[(size_t)c * K + k] += pi;
      }
      if (win) lp += -(o.y[label] - mx - log(se));
    }
    o.loss[c] += lp;
  }
  if (n.reg_mode == 1) {
    // moving-average regulariser's loss of step t (eq. ema-rate)
    double acc = 0.0;
    for (uint32_t j = tid; j < n.J; j += blockDim.x) {
      const double df = (double)o.fh[(size_t)t * n.Jp + j] - n.f_target;
      acc += df * df;
    }
    red[tid] = acc;
    __syncthreads();
    for (uint32_t sz = 128; sz > 0; sz >>= 1) {
      if (tid < sz) red[tid] += red[tid + sz];
      __syncthreads();
    }
    if (tid == 0) o.loss[c] += 0.5 * n.c_reg * red[0];
  }
}

// Fixed-order reduction of the trial-chunk partial sums into (gs, gc).
template <typename real>
__global__ __launch_bounds__(256) void k_synapse_reduce(DevNet<real> n, uint32_t nchunk, const real *partial) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n.S; q += (uint64_t)gridDim.x * blockDim.x) {
    real gs = n.g_fresh ? (real)0 : n.gs[q], gc = n.g_fresh ? (real)0 : n.gc[q];
    for (uint32_t c = 0; c < nchunk; ++c) kahan_add(gs, gc, partial[(size_t)c * n.S + q]);
    n.gs[q] = gs;
    n.gc[q] = gc;
  }
}

// Output-synapse gradients of the batch's trials, summed in trial order.
template <typename real>
__global__ __launch_bounds__(256) void k_output_reduce(DevNet<real> n) {
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  const size_t total = (size_t)n.K * n.Jp;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    real s = n.gos[i], c = n.goc[i];
    for (uint32_t b = 0; b < ntr; ++b) kahan_add(s, c, n.gout_b[(size_t)b * total + i]);
    n.gos[i] = s;
    n.goc[i] = c;
  }
}

// ----------------------------------------------------------------- optimiser

__device__ inline void opt_step(double &w, double G, int opt, double eta, double eta_t, double b1,
                                double b2, double eps, double &m, double &v) {
  if (opt == 0) {
    w = w - eta * G;
  } else {
    m = b1 * m + (1.0 - b1) * G;
    v = b2 * v + (1.0 - b2) * G * G;
    w = w - eta_t * m / (sqrt(v) + eps);
  }
}

template <typename real>
__global__ __launch_bounds__(256) void k_apply_syn(DevNet<real> n, uint64_t S, double n_trials, int opt,
                                                   double eta, double eta_t, double b1, double b2, double eps) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < S; q += (uint64_t)gridDim.x * blockDim.x) {
    const double G = ((double)n.gs[q] + (double)n.gc[q]) / n_trials;
    double w = (double)n.tm_w[q], m = 0.0, v = 0.0;
    if (opt == 1) {
      m = (double)n.adam_m[q];
      v = (double)n.adam_v[q];
    }
    opt_step(w, G, opt, eta, eta_t, b1, b2, eps, m, v);
    if (opt == 1) {
      n.adam_m[q] = (real)m;
      n.adam_v[q] = (real)v;
    }
    n.tm_w[q] = (real)w;
    if (n.dlw) *reinterpret_cast<real *>(n.dlw + n.tm_dpos[q]) = (real)w;
    n.gs[q] = (real)0;
    n.gc[q] = (real)0;
  }
}

template <typename real>
__global__ __launch_bounds__(256) void k_apply_out(DevNet<real> n, double n_trials, int opt, double eta,
                                                   double eta_t, double b1, double b2, double eps) {
  const size_t total = (size_t)n.K * n.Jp;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    if (i % n.Jp >= n.J) continue;
    const double G = ((double)n.gos[i] + (double)n.goc[i]) / n_trials;
    double w = (double)n.w_out[i], m = 0.0, v = 0.0;
    if (opt == 1) {
      m = (double)n.adam_mo[i];
      v = (double)n.adam_vo[i];
    }
    opt_step(w, G, opt, eta, eta_t, b1, b2, eps, m, v);
    if (opt == 1) {
      n.adam_mo[i] = (real)m;
      n.adam_vo[i] = (real)v;
    }
    n.w_out[i] = (real)w;
    n.gos[i] = (real)0;
    n.goc[i] = (real)0;
  }
}

// Bound on the input current of one step: every synapse delivers at most
// one spike per step, so |I_j^t| <= sum of |w| over j's incoming synapses.
// One wavefront per target (coalesced over its target-major row); the
// maximum over targets, slightly enlarged to cover the rounding of the sum,
// goes to *l1max (positive floats order like their bit patterns).
// Weight update with scatter delivery on networks whose rows are dense
// within a tile (many synapses per source and tile): an explicit blocked
// transposition through LDS.  Block c owns the synapses from sources
// s0..s1-1 into the targets of tile k.  Source rows are sorted by target,
// so these are one contiguous segment of each source row (tseg) and one
// segment of the delivery table (dseg); target rows are sorted by source,
// so they are also one contiguous run of each target row (starting at
// trs[c][t]).  The block reads the runs' gradients (Kahan pairs) and their
// source-major positions, puts each averaged gradient into LDS at its place
// in the block's source-major order, and then updates the weights of the
// delivery table segment by segment: both sides of HBM are read and written
// in runs, with no scattered words.  It
// also sums |w| per target of the tile in LDS (fixed point, each term
// rounded up, so the sum bounds the input current of any step) and adds
// the sums to tsum; k_bound_max turns the largest into *l1max.
// UPDATE = false only recomputes the bound.
template <typename real, bool UPDATE>
__global__ __launch_bounds__(1024) void k_apply_blk(DevNet<real> n, uint32_t n_ach, double n_trials, int opt,
                                                    double eta, double eta_t, double b1, double b2, double eps) {
  constexpr uint32_t NT = 1024;
  constexpr uint32_t PER_S = kApplySrc / NT;
  constexpr uint32_t PER_T = kApplyMaxTile / NT;
  constexpr uint32_t WPR = sizeof(real) / 4;  // words per weight
  __shared__ uint32_t pre[kApplySrc + 1];
  __shared__ uint32_t seg0[kApplySrc];  // first synapse (source-major index) of each source's segment
  __shared__ uint32_t dw0[kApplySrc];   // word index of each source's segment in the delivery table
  __shared__ uint32_t wsum[17];
  extern __shared__ __align__(16) unsigned char apl_smem[];
  const uint32_t TS = n.TS;
  unsigned long long *tsl = reinterpret_cast<unsigned long long *>(apl_smem);  // [TS]
  uint32_t *tpre = reinterpret_cast<uint32_t *>(tsl + TS);                     // [TS + 1]
  uint32_t *tr0 = tpre + TS + 1;                                               // [TS]
  real *gbuf = reinterpret_cast<real *>(apl_smem + (size_t)TS * 16 + 16);       // [kApplySyn(real)]
  const uint32_t tid = threadIdx.x, c = blockIdx.x;
  const uint32_t k = n.ach[3 * c], s0 = n.ach[3 * c + 1], s1 = n.ach[3 * c + 2];
  const uint32_t nsrc = s1 - s0, j0 = k * TS;
  const bool last_of_tile = c + 1 >= n_ach || n.ach[3 * (c + 1)] != k;
  for (uint32_t i = tid; i < TS; i += NT) tsl[i] = 0ull;
  // source-major side: the segment of each source, scanned
  uint32_t len[PER_S], lo[PER_S], dw[PER_S], sum = 0;
#pragma unroll
  for (uint32_t u = 0; u < PER_S; ++u) {
    const uint32_t i = tid * PER_S + u;
    len[u] = 0;
    lo[u] = 0;
    dw[u] = 0;
    if (i < nsrc) {
      lo[u] = n.tseg[(size_t)(s0 + i) * (n.KT + 1) + k];
      const uint2 sg = n.dseg[(size_t)(s0 + i) * n.KT + tile_rank(k, n.KT)];
      dw[u] = sg.x;
      len[u] = sg.y;
    }
    sum += len[u];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, wsum, &total);
#pragma unroll
  for (uint32_t u = 0; u < PER_S; ++u) {
    const uint32_t i = tid * PER_S + u;
    if (i < nsrc) {
      pre[i] = run;
      seg0[i] = lo[u];
      dw0[i] = dw[u];
    }
    run += len[u];
  }
  if (tid == 0) pre[nsrc] = total;
  if constexpr (UPDATE) {
    __syncthreads();  // the scan's partial sums are reused below
    // target-major side: the run of each target, scanned
    uint32_t tl[PER_T], t0[PER_T], tsum_ = 0;
#pragma unroll
    for (uint32_t u = 0; u < PER_T; ++u) {
      const uint32_t t = tid * PER_T + u, j = j0 + t;
      tl[u] = 0;
      t0[u] = 0;
      if (t < TS && j < n.J) {
        const uint32_t r0 = n.trs[(size_t)c * TS + t];
        const uint32_t r1 = last_of_tile ? n.tm_ptr[j + 1] : n.trs[(size_t)(c + 1) * TS + t];
        t0[u] = r0;
        tl[u] = r1 - r0;
      }
      tsum_ += tl[u];
    }
    uint32_t ttot;
    uint32_t trun = block_exclusive_scan(tsum_, wsum, &ttot);
#pragma unroll
    for (uint32_t u = 0; u < PER_T; ++u) {
      const uint32_t t = tid * PER_T + u;
      if (t < TS) {
        tpre[t] = trun;
        tr0[t] = t0[u];
      }
      trun += tl[u];
    }
    if (tid == 0) tpre[TS] = ttot;
    __syncthreads();
    // gradients in target-major runs -> LDS in the block's source-major
    // order, GB elements per thread at a time so that their loads are in
    // flight together (an element beyond the runs repeats element i0)
    constexpr uint32_t GB = 8;
    for (uint32_t i0 = tid; i0 < ttot; i0 += GB * NT) {
      uint32_t qv[GB];
#pragma unroll
      for (uint32_t u = 0; u < GB; ++u) {
        const uint32_t i = min(i0 + u * NT, ttot - 1);
        uint32_t a = 0, b = TS;  // tpre[a] <= i < tpre[b]
        while (b - a > 1) {
          const uint32_t m = (a + b) >> 1;
          if (tpre[m] <= i) a = m; else b = m;
        }
        qv[u] = tr0[a] + (i - tpre[a]);
      }
      real gsv[GB], gcv[GB];
      uint16_t lv[GB];
#pragma unroll
      for (uint32_t u = 0; u < GB; ++u) {
        gsv[u] = n.gs[qv[u]];
        gcv[u] = n.gc[qv[u]];
        lv[u] = n.tm_loc[qv[u]];  // its place in the block's segments (built at create)
      }
#pragma unroll
      for (uint32_t u = 0; u < GB; ++u) {
        const uint32_t local = lv[u];
        if (i0 + u * NT < ttot && local < total)
          gbuf[local] = (real)(((double)gsv[u] + (double)gcv[u]) / n_trials);
      }
    }
  }
  __syncthreads();
  // source-major side: update the weights segment by segment, BU elements
  // per thread at a time with all their loads issued before their stores
  // (vector memory operations complete in order, so a load issued after a
  // store waits for it); an element beyond the block repeats element i0's
  // addresses and is not written
  constexpr uint32_t BU = 4;
  const uint16_t *o16 = reinterpret_cast<const uint16_t *>(n.dlw);
  for (uint32_t i0 = tid; i0 < total; i0 += BU * NT) {
    uint32_t qv[BU], wv[BU], ov[BU];
#pragma unroll
    for (uint32_t u = 0; u < BU; ++u) {
      const uint32_t i = min(i0 + u * NT, total - 1);
      uint32_t a = 0, b = nsrc;  // pre[a] <= i < pre[b]
      while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (pre[m] <= i) a = m; else b = m;
      }
      const uint32_t rel = i - pre[a], L = pre[a + 1] - pre[a];
      qv[u] = seg0[a] + rel;
      wv[u] = dw0[a] + rel * WPR;
      ov[u] = 2 * dw0[a] + L * (sizeof(real) / 2) + rel;
    }
#pragma unroll
    for (uint32_t u = 1; u < BU; ++u)
      if (i0 + u * NT >= total) {
        qv[u] = qv[0];
        wv[u] = wv[0];
        ov[u] = ov[0];
      }
    real rw[BU], mv[BU], vv[BU];
    uint32_t ro[BU];
#pragma unroll
    for (uint32_t u = 0; u < BU; ++u) {
      rw[u] = *reinterpret_cast<const real *>(n.dlw + wv[u]);
      ro[u] = o16[ov[u]];
    }
    if (UPDATE && opt == 1) {
#pragma unroll
      for (uint32_t u = 0; u < BU; ++u) {
        mv[u] = n.adam_m[qv[u]];
        vv[u] = n.adam_v[qv[u]];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < BU; ++u) {
      const uint32_t i = i0 + u * NT;
      if (i >= total) break;
      const uint32_t q = qv[u];
      double w = (double)rw[u];
      if constexpr (UPDATE) {
        const double G = (double)gbuf[i];
        double m = 0.0, v = 0.0;
        if (opt == 1) {
          m = (double)mv[u];
          v = (double)vv[u];
        }
        opt_step(w, G, opt, eta, eta_t, b1, b2, eps, m, v);
        if (opt == 1) {
          n.adam_m[q] = (real)m;
          n.adam_v[q] = (real)v;
        }
        const real wr = (real)w;
        *reinterpret_cast<real *>(n.dlw + wv[u]) = wr;
        w = (double)wr;
      }
      // the target in the tile: the ring offset o = d * TS + t
      const uint32_t o = ro[u];
      const uint32_t t = o - TS * (uint32_t)(((uint64_t)o * n.ts_magic) >> 32);
      const double aw = fabs(w);
      if (aw < kBoundMaxW) {
        atomicAdd(&tsl[t], (unsigned long long)ceil(aw * kBoundScale));
      } else {
        atomicOr(&n.tsum[j0 + t], 1ull << 63);  // saturated: reported as an out-of-range bound
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < TS && j0 + i < n.Jp; i += NT)
    if (tsl[i]) atomicAdd(&n.tsum[j0 + i], tsl[i]);
}

// *l1max = the largest per-target bound (with a margin for the conversion),
// and tsum cleared for the next update.
template <typename real>
__global__ __launch_bounds__(256) void k_bound_max(DevNet<real> n) {
  float mx = 0.f;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n.J; j += gridDim.x * blockDim.x) {
    const unsigned long long t = n.tsum[j];
    n.tsum[j] = 0ull;
    const float l = (t >> 63) ? 0x1p60f : (float)((double)t / kBoundScale * 1.001);
    mx = fmaxf(mx, l);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63u) == 0 && mx > 0.f) atomicMax(n.l1max, __float_as_uint(mx));
}

template <typename real>
__global__ __launch_bounds__(256) void k_input_bound(DevNet<real> n) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = (gridDim.x * blockDim.x) >> 6;
  float mx = 0.f;
  for (uint32_t j = w0; j < n.J; j += nwv) {
    double acc = 0.0;
    for (uint32_t q = n.tm_ptr[j] + lane; q < n.tm_ptr[j + 1]; q += 64) acc += fabs((double)n.tm_w[q]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    mx = fmaxf(mx, (float)(acc * 1.001));
  }
  if (lane == 0 && mx > 0.f) atomicMax(n.l1max, __float_as_uint(mx));
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
inline uint32_t grid_for(uint64_t work, uint32_t block, uint32_t cap = 8192) {
  const uint32_t g = cdiv(work ? work : 1, block);
  return g < cap ? g : cap;
}

}  // namespace

// ----------------------------------------------------------------- launchers

template <typename real>
void Launch<real>::stage_inputs(const DevNet<real> &n, uint32_t ntr, uint64_t nsp, bool check_order,
                                hipStream_t s) {
  if (nsp > 0)
    k_stage_in_bits<real><<<grid_for(nsp, 256), 256, 0, s>>>(n, ntr, nsp, check_order ? 1 : 0);
  k_stage_in_step_ptr<real><<<dim3(cdiv(n.Tcap + 1, 256), n.Bcap), 256, 0, s>>>(n);
  if (n.I > 0) k_stage_in_lists<real><<<dim3(cdiv(n.Iw, 4), n.Bcap), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::stage_forced(const DevNet<real> &n, uint32_t ntr, uint64_t nf, hipStream_t s) {
  if (nf > 0) k_stage_forced<real><<<grid_for(nf, 256), 256, 0, s>>>(n, ntr, nf);
}

template <typename real>
void Launch<real>::rec_lists(const DevNet<real> &n, uint32_t ntr, hipStream_t s) {
  if (n.J > 0) k_stage_rec_lists<real><<<dim3(cdiv(n.Jw, 4), ntr), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::neuron_gather(const DevNet<real> &n, uint32_t off, bool forced, hipStream_t s) {
  const dim3 grid(cdiv(n.Jp, 256), n.Bcap);
  if (forced) k_neuron_gather<real, true><<<grid, 256, 0, s>>>(n, off);
  else k_neuron_gather<real, false><<<grid, 256, 0, s>>>(n, off);
}

template <typename real>
size_t Launch<real>::tile_smem(uint32_t TS, uint32_t R, uint32_t ring_bytes, uint32_t ptab_cap) {
  return (size_t)R * TS * ring_bytes + (size_t)2 * TS * sizeof(real) + (size_t)(TS / 64) * 8 +
         ((TS / 64 + 2) & ~1u) * 4 + (size_t)ptab_cap * 8 + TS + (size_t)(TS / 64) * 8 + 64;
}

// The forward kernels of a precision and ring element, one per delivery variant.
template <typename real, typename ring_t>
struct FwdKernels {
  template <bool F>
  static const void *get_v(uint32_t v) {
    switch (v) {
      case 1: return reinterpret_cast<const void *>(&k_forward_tiled<real, ring_t, F, 1>);
      case 2: return reinterpret_cast<const void *>(&k_forward_tiled<real, ring_t, F, 2>);
      case 3: return reinterpret_cast<const void *>(&k_forward_tiled<real, ring_t, F, 3>);
      case 4: return reinterpret_cast<const void *>(&k_forward_tiled<real, ring_t, F, 4>);
      default: return reinterpret_cast<const void *>(&k_forward_tiled<real, ring_t, F, 0>);
    }
  }
  static const void *get(bool forced, uint32_t v) { return forced ? get_v<true>(v) : get_v<false>(v); }
  template <bool F>
  static void launch_v(const DevNet<real> &n, uint32_t nsteps, uint32_t b0, uint32_t v, uint32_t grid,
                       uint32_t block, size_t smem, hipStream_t s) {
    switch (v) {
      case 1: k_forward_tiled<real, ring_t, F, 1><<<grid, block, smem, s>>>(n, nsteps, b0); break;
      case 2: k_forward_tiled<real, ring_t, F, 2><<<grid, block, smem, s>>>(n, nsteps, b0); break;
      case 3: k_forward_tiled<real, ring_t, F, 3><<<grid, block, smem, s>>>(n, nsteps, b0); break;
      case 4: k_forward_tiled<real, ring_t, F, 4><<<grid, block, smem, s>>>(n, nsteps, b0); break;
      default: k_forward_tiled<real, ring_t, F, 0><<<grid, block, smem, s>>>(n, nsteps, b0); break;
    }
  }
  static void launch(const DevNet<real> &n, uint32_t nsteps, uint32_t b0, bool forced, uint32_t v, uint32_t grid,
                     uint32_t block, size_t smem, hipStream_t s) {
    if (forced) launch_v<true>(n, nsteps, b0, v, grid, block, smem, s);
    else launch_v<false>(n, nsteps, b0, v, grid, block, smem, s);
  }
};

template <typename real>
const void *fwd_kernel(uint32_t ring_bytes, bool forced, uint32_t v) {
  if constexpr (sizeof(real) == 8) return FwdKernels<double, double>::get(forced, v);
  else return FwdKernels<float, int32_t>::get(forced, v);
}

template <typename real>
hipError_t Launch<real>::allow_smem(size_t smem, uint32_t ring_bytes) {
  hipError_t e = hipSuccess;
  for (uint32_t v = 0; v < kFwdVariants && e == hipSuccess; ++v)
    for (int f = 0; f < 2 && e == hipSuccess; ++f)
      e = hipFuncSetAttribute(fwd_kernel<real>(ring_bytes, f == 1, v), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)smem);
  return e;
}

template <typename real>
hipError_t Launch<real>::resident(uint32_t block, size_t smem, uint32_t ring_bytes, int *per_cu) {
  // the variant with the fewest resident workgroups decides
  int best = 1 << 30;
  for (uint32_t v = 0; v < kFwdVariants; ++v) {
    int pc = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, fwd_kernel<real>(ring_bytes, false, v), (int)block, smem);
    if (e != hipSuccess) return e;
    best = pc < best ? pc : best;
  }
  *per_cu = best;
  return hipSuccess;
}

// The trials' tiles wait for each other within a trial, so every launch holds
// only as many trials as the device keeps resident together (sh.fwd_trials);
// larger batches run in consecutive launches of such chunks.
template <typename real>
void Launch<real>::forward_tiled(const DevNet<real> &n, uint32_t nsteps, bool forced, const Shapes &sh, size_t smem,
                                 hipStream_t s) {
  const uint32_t v = sh.fwd_variant < kFwdVariants ? sh.fwd_variant : 0u;
  const uint32_t per = sh.fwd_trials ? sh.fwd_trials : n.Bcap;
  for (uint32_t b0 = 0; b0 < n.Bcap; b0 += per) {
    const uint32_t grid = (b0 + per <= n.Bcap ? per : n.Bcap - b0) * n.KT;
    if constexpr (sizeof(real) == 8)
      FwdKernels<double, double>::launch(n, nsteps, b0, forced, v, grid, sh.tile_block, smem, s);
    else
      FwdKernels<float, int32_t>::launch(n, nsteps, b0, forced, v, grid, sh.tile_block, smem, s);
  }
}

template <typename real>
void Launch<real>::readout(const DevNet<real> &n, hipStream_t s) {
  k_readout_sums<real><<<dim3(cdiv(n.Tcap, 4), n.Bcap), 256, 0, s>>>(n);
  k_readout_scan<real><<<n.Bcap, 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::adjoint(const DevNet<real> &n, const Shapes &sh, hipStream_t s) {
  const uint32_t bd = sh.adj_block;
  const size_t smem = (size_t)n.K * bd * 8 + 16 * (size_t)n.K * 8 + (size_t)bd * 17 * sizeof(real);
  const dim3 grid(n.Jp / bd + (n.Jp % bd ? 1 : 0), n.Bcap);
  if (n.reset_mode == 1 || n.reg_mode == 1) k_adjoint<real, true><<<grid, bd, smem, s>>>(n);
  else k_adjoint<real, false><<<grid, bd, smem, s>>>(n);
}

template <typename real>
void Launch<real>::synapse(const DevNet<real> &n, const Shapes &sh, uint32_t n_trials, real *partial, hipStream_t s) {
  const uint32_t nchunk = (n_trials + sh.ginst - 1) / sh.ginst;
  const uint32_t N = nchunk * n.NS, nblk = (N + kScanItems - 1) / kScanItems;
  k_pack_scan_local<real><<<nblk, 1024, 0, s>>>(n, sh.ginst, N);
  k_pack_scan_blocks<real><<<1, 1024, 0, s>>>(n, nblk);
  k_pack_fill<real><<<cdiv(N, 256), 256, 0, s>>>(n, sh.ginst, N, nblk);
  const size_t smem = ((size_t)sh.ginst * n.Ts + n.R) * sizeof(real);
  const dim3 grid(n.J * nchunk);
  switch (sh.syn_var) {
    case 1: k_synapse<real, syn_pre_of(1), syn_batch_of(1)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    case 2: k_synapse<real, syn_pre_of(2), syn_batch_of(2)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    case 3: k_synapse<real, syn_pre_of(3), syn_batch_of(3)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    case 4: k_synapse<real, syn_pre_of(4), syn_batch_of(4)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    case 5: k_synapse<real, syn_pre_of(5), syn_batch_of(5)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    case 6: k_synapse<real, syn_pre_of(6), syn_batch_of(6)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
    default: k_synapse<real, syn_pre_of(0), syn_batch_of(0)><<<grid, sh.syn_block, smem, s>>>(n, sh.ginst, nchunk, partial); break;
  }
  if (nchunk > 1) k_synapse_reduce<real><<<grid_for(n.S, 256, 16384), 256, 0, s>>>(n, nchunk, partial);
}

template <typename real>
void Launch<real>::time_driven(const DevNet<real> &n, const Shapes &sh, uint32_t n_trials, real *L, real *partial,
                               hipStream_t s) {
  const uint32_t nchunk = (n_trials + sh.ginst - 1) / sh.ginst;
  k_learning_signal<real><<<grid_for((uint64_t)n_trials * n.Jp * n.Tp, 256, 16384), 256, 0, s>>>(n, L);
  // one workgroup per target when the chunk's psi and L rows fit LDS
  const size_t smem = (size_t)2 * sh.ginst * n.Tp * sizeof(real);
  if (n.S > 0 && smem <= (size_t)160 * 1024) {
    if (smem > (size_t)64 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_td_target<real>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    // psi transposed into the arrival archive's buffer, which the
    // time-driven gradient does not use
    k_transpose_psi<real><<<dim3((n.Tp + 63) / 64, (n.Jp + 63) / 64, n_trials), 256, 0, s>>>(n, n.phi);
    k_td_target<real><<<dim3(n.J, nchunk), 256, smem, s>>>(n, L, n.phi, sh.ginst, nchunk, partial);
  } else if (n.S > 0) {
    k_td_synapse<real><<<cdiv(n.S * nchunk, 256), 256, 0, s>>>(n, L, sh.ginst, nchunk, partial);
  }
  if (nchunk > 1 && n.S > 0) k_synapse_reduce<real><<<grid_for(n.S, 256, 16384), 256, 0, s>>>(n, nchunk, partial);
  k_td_output<real><<<grid_for((uint64_t)n_trials * n.K * n.Jp, 256, 16384), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::output_reduce(const DevNet<real> &n, hipStream_t s) {
  k_output_reduce<real><<<grid_for((uint64_t)n.K * n.Jp, 256, 2048), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::apply(const DevNet<real> &n, uint64_t S, double n_trials, int opt, double eta,
                         double eta_t, double b1, double b2, double eps, hipStream_t s) {
  if (S > 0) k_apply_syn<real><<<grid_for(S, 256, 16384), 256, 0, s>>>(n, S, n_trials, opt, eta, eta_t, b1, b2, eps);
  k_apply_out<real><<<grid_for((uint64_t)n.K * n.Jp, 256, 2048), 256, 0, s>>>(n, n_trials, opt, eta, eta_t, b1, b2, eps);
}

// dynamic LDS of k_apply_blk: bound sums, target scan, run starts, and the
// block's gradients (kApplySyn * 4 bytes: kApplySyn FP32 or half as many FP64)
static size_t apply_blk_smem(uint32_t TS) { return (size_t)TS * 16 + 16 + (size_t)kApplySyn * 4; }

template <typename real>
static void launch_apply_blk(const DevNet<real> &n, uint32_t n_ach, bool update, double n_trials, int opt,
                             double eta, double eta_t, double b1, double b2, double eps, hipStream_t s) {
  const size_t smem = apply_blk_smem(n.TS);
  (void)hipMemsetAsync(n.l1max, 0, sizeof(uint32_t), s);
  if (n_ach) {
    if (update) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_apply_blk<real, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      k_apply_blk<real, true><<<n_ach, 1024, smem, s>>>(n, n_ach, n_trials, opt, eta, eta_t, b1, b2, eps);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_apply_blk<real, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      k_apply_blk<real, false><<<n_ach, 1024, smem, s>>>(n, n_ach, n_trials, opt, eta, eta_t, b1, b2, eps);
    }
  }
  k_bound_max<real><<<grid_for(n.J, 256, 1024), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::apply_blocked(const DevNet<real> &n, uint32_t n_ach, uint64_t S, double n_trials, int opt,
                                 double eta, double eta_t, double b1, double b2, double eps, hipStream_t s) {
  // (the gradient pairs are not cleared: the first training batch after an
  // update writes them instead of adding to them, see g_fresh)
  (void)S;
  launch_apply_blk(n, n_ach, true, n_trials, opt, eta, eta_t, b1, b2, eps, s);
  k_apply_out<real><<<grid_for((uint64_t)n.K * n.Jp, 256, 2048), 256, 0, s>>>(n, n_trials, opt, eta, eta_t, b1, b2, eps);
}

template <typename real>
void Launch<real>::online_fill(const DevNet<real> &n, bool to_records, hipStream_t s) {
  k_online_fill<real><<<grid_for(n.S, 256, 16384), 256, 0, s>>>(n, to_records ? 1 : 0);
}

template <typename real>
void Launch<real>::online_step(const DevNet<real> &n, const OnlineRun<real> &o, uint32_t t, bool forced,
                               hipStream_t s) {
  k_online_syn<real><<<(n.J + 3) / 4, 256, 0, s>>>(n, o, t);
  const uint32_t blocks = n.Jp / 256 + (n.Jp % 256 ? 1 : 0);
  if (forced) k_online_neuron<real, true><<<blocks, 256, 0, s>>>(n, o, t);
  else k_online_neuron<real, false><<<blocks, 256, 0, s>>>(n, o, t);
  const uint32_t KB = n.K < 256 ? n.K : 256;
  k_online_out_syn<real><<<(n.Jw + 256 / KB - 1) / (256 / KB), 256, 0, s>>>(n, o, t);
  k_online_readout<real><<<1, 256, 0, s>>>(n, o, t);
  k_online_learn<real><<<(n.J + 255) / 256, 256, 0, s>>>(n, o, t);
}

template <typename real>
size_t Launch<real>::apply_blocked_smem(uint32_t TS) {
  return apply_blk_smem(TS) + sizeof(uint32_t) * (3 * kApplySrc + 1 + 17);
}

template <typename real>
void Launch<real>::input_bound_blocked(const DevNet<real> &n, uint32_t n_ach, hipStream_t s) {
  launch_apply_blk(n, n_ach, false, 1.0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, s);
}

template <typename real>
void Launch<real>::input_bound(const DevNet<real> &n, hipStream_t s) {
  (void)hipMemsetAsync(n.l1max, 0, sizeof(uint32_t), s);
  k_input_bound<real><<<grid_for((uint64_t)n.J * 64, 256, 4096), 256, 0, s>>>(n);
}

void launch_advance(uint32_t *ctl, uint32_t by, hipStream_t s) { k_advance<<<1, 64, 0, s>>>(ctl, by); }

// ------------------------------------------------- no-allocation staging
// Staging memory of the no-allocation batch call: the copies of a
// host-memory batch's arrays, which the staging and readout kernels read.
// Each GPU the library runs on holds its own copy of this array until the
// process ends; every call on one GPU shares it, so such calls that overlap
// on one GPU race.  The name is a host-side stand-in in host code: only the
// address from hipGetSymbolAddress, taken with the device current, is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void *scratch_address(int device, hipError_t *err) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *err = e;
      return nullptr;
    }
    addr[device] = p;
  }
  *err = hipSuccess;
  return addr[device];
}

uint32_t fwd_variant_piece(uint32_t v) { return fwd_piece(v); }
uint32_t syn_variant_pre(uint32_t v) { return syn_pre_of(v); }
uint32_t syn_variant_batch(uint32_t v) { return syn_batch_of(v); }
static_assert(kNumSynVariants == kSynVariants, "synapse variant count");
uint32_t fwd_variant_unroll(uint32_t v) { return fwd_unroll(v); }
static_assert(kNumFwdVariants == kFwdVariants, "variant count");

template struct Launch<float>;
template struct Launch<double>;

}  // namespace eprop
