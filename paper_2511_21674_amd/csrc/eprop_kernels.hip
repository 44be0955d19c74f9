// HIP kernels of the event-driven e-prop library (gfx950, wave64).
//
// Within one iteration the weights are fixed and the gradient of a sample
// is formed from the sample's archived history (paper, Results: the
// event-driven implementation computes the gradient at the first spike
// after each sample from the archived postsynaptic history).  The path is:
//
//   forward, per step t     k_neuron  (time-driven neuron update, eq. lif_update,
//                                      eq. spike-threshold-adaptation, surrogate)
//                           k_deliver (spike delivery into delay rings)
//   after the sample        k_readout_sums, k_readout_scan (eq. leaky_integrator,
//                                      error signal, loss; backward filter of E)
//                           k_adjoint (per-neuron arrival archive phi)
//                           k_synapse (event-driven synapse gradient)
//                           k_output_reduce
//   end of iteration        k_apply_syn, k_apply_out (GD or Adam)
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

// Per-channel input spike-time lists, ascending, from the bitsets.
template <typename real>
__global__ __launch_bounds__(256) void k_stage_in_lists(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n.I) return;
  const uint32_t T = n.T[b];
  const uint64_t *bits = n.in_bits + (size_t)b * n.Tcap * n.Iw + (i >> 6);
  uint16_t *out = n.spk_t + (size_t)b * n.spk_stride + (size_t)i * n.Tcap;
  uint32_t c = 0;
  for (uint32_t s = 0; s < T; ++s)
    if ((bits[(size_t)s * n.Iw] >> (i & 63u)) & 1ull) out[c++] = (uint16_t)s;
  n.spk_cnt[(size_t)b * n.NS + i] = c;
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

// Neuron update at step t = ctl[T0] + off for every (trial, neuron).
// GATHER sums the arriving synapses of each target in ascending source
// order (inputs first); otherwise the input is read from the delay ring.
// The expression order matches the reference definition, so FP64 with
// GATHER reproduces it bit for bit.
template <typename real, bool GATHER, bool FORCED>
__global__ __launch_bounds__(256) void k_neuron(DevNet<real> n, uint32_t off) {
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
  if constexpr (GATHER) {
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
  } else {
    real *slot = n.ring + ((size_t)b * n.R + t % n.R) * n.Jp + j;
    I = *slot;
    *slot = (real)0;
  }

  const uint8_t st = n.nst[sidx];
  uint32_t refr = st & 0x7Fu;
  const real zprev = (st & 0x80u) ? (real)1 : (real)0;
  const real beta = n.beta_j[j];
  real A = n.v_th;
  if (beta != (real)0) {  // LIF: v_th + 0 * a == v_th
    real a = n.a[sidx];
    a = n.rho * a + zprev;
    n.a[sidx] = a;
    A = n.v_th + beta * a;
  }
  real v = n.v[sidx];
  v = n.alpha * v + I - zprev * A;
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
  n.v[sidx] = v;
  n.nst[sidx] = (uint8_t)(refr | (z ? 0x80u : 0u));
  n.psi[((size_t)b * (n.Tcap + 1) + t) * n.Jp + j] = ps;

  const uint64_t word = __ballot(z);
  const uint32_t lane = lane_id();
  uint32_t base = 0;
  if (lane == 0) {
    n.rec_bits[((size_t)b * (n.Tcap + 1) + t) * n.Jw + (j >> 6)] = word;
    if (word) {
      const uint32_t c = (uint32_t)__popcll(word);
      base = atomicAdd(&n.rec_cnt[(size_t)b * (n.Tcap + 1) + t], c);
      atomicAdd(&n.cnt[CNT_REC_SPIKES], (unsigned long long)c);
    }
  }
  base = (uint32_t)__shfl((int)base, 0);
  if (z) {
    const uint32_t pos = base + (uint32_t)__popcll(word & ((1ull << lane) - 1ull));
    n.rec_list[((size_t)b * 2 + (t & 1u)) * n.Jp + pos] = j;
    const size_t ci = (size_t)b * n.NS + n.I + j;
    const uint32_t c = n.spk_cnt[ci];
    n.spk_t[(size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Tcap + c] = (uint16_t)t;
    n.spk_cnt[ci] = c + 1;
  }
}

// Spike delivery for the spikes emitted at step t = ctl[T0] + off: input
// spikes of that step and recurrent spikes of that step.  One wavefront per
// spiking source walks its outgoing synapses and adds the weight into the
// target's ring slot for step t + D (only arrivals within the trial).
template <typename real>
__global__ __launch_bounds__(256) void k_deliver(DevNet<real> n, uint32_t off, const uint32_t *const *in_src_pp) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t t = n.ctl[CTL_T0] + off;
  const uint32_t Tb = n.T[b];
  if (t >= Tb) return;
  const uint64_t *isp = n.in_step_ptr + (size_t)b * (n.Tcap + 1);
  const uint64_t in_lo = isp[t], in_hi = isp[t + 1];
  const uint32_t n_in = in_hi > in_lo ? (uint32_t)(in_hi - in_lo) : 0u;
  const uint32_t n_rec = t >= 1 ? n.rec_cnt[(size_t)b * (n.Tcap + 1) + t] : 0u;
  const uint32_t total = n_in + n_rec;
  const uint32_t lane = lane_id();
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t *in_src = *in_src_pp;
  const uint32_t *rl = n.rec_list + ((size_t)b * 2 + (t & 1u)) * n.Jp;
  real *ring = n.ring + (size_t)b * n.R * n.Jp;
  for (uint32_t item = wave; item < total; item += nwaves) {
    const uint32_t src = item < n_in ? in_src[in_lo + item] : n.I + rl[item - n_in];
    const uint32_t q1 = n.sm_ptr[src + 1];
    for (uint32_t q = n.sm_ptr[src] + lane; q < q1; q += 64) {
      const uint32_t pk = n.sm_syn[q];
      const uint32_t ta = t + (pk >> 24);
      if (ta <= Tb) atomicAdd(&ring[(size_t)(ta % n.R) * n.Jp + (pk & 0xFFFFFFu)], n.sm_w[q]);
    }
  }
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

// Per trial (one block of 256): readout recursion y^t = kappa y^{t-1} + ysum^t,
// error signal and loss (window-gated), prediction, and the backward filter
// Ebar^t = E^t + kappa Ebar^{t+1}.  All FP64.
template <typename real>
__global__ __launch_bounds__(256) void k_readout_scan(DevNet<real> n) {
  const uint32_t b = blockIdx.x;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t T = n.T[b], K = n.K, tid = threadIdx.x;
  const size_t rs = (size_t)(n.Tcap + 2) * K;
  double *ysum = n.ysum + b * rs, *y = n.y + b * rs, *err = n.err + b * rs, *ebar = n.ebar + b * rs;
  const double kap = n.kappa_d;
  for (uint32_t k = tid; k < K; k += blockDim.x) {
    double yy = 0.0;
    for (uint32_t t = 1; t <= T; ++t) {
      yy = kap * yy + ysum[(size_t)t * K + k];
      y[(size_t)t * K + k] = yy;
    }
  }
  __syncthreads();
  double lp = 0.0;
  const uint32_t label = n.loss == 1 ? n.label[b] : 0u;
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
  __shared__ double red[256];
  __shared__ double psum[64];
  red[tid] = lp;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  for (uint32_t k = tid; k < K; k += blockDim.x) {
    double eb = 0.0;
    for (uint32_t t = T; t >= 1; --t) {
      eb = err[(size_t)t * K + k] + kap * eb;
      ebar[(size_t)t * K + k] = eb;
    }
    if (n.loss == 1 && k < 64) {
      double s = 0.0;
      for (uint32_t t = 1; t <= T; ++t) s += ysum[(size_t)t * K + k];
      psum[k] = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    n.loss_out[b] = red[0];
    uint32_t best = 0;
    if (n.loss == 1)
      for (uint32_t k = 1; k < K && k < 64; ++k)
        if (psum[k] > psum[best]) best = k;
    n.pred_out[b] = best;
  }
}

// ----------------------------------------------------------------- gradient

// Per (trial, neuron), backward over the trial: learning signal of the
// filtered errors Lambda^t = sum_k B_jk Ebar_k^t, adjoint recursion of the
// eligibility vector (FP64), archive phi[b][j][t] = mu^t[0]; then the
// neuron's output-synapse gradient sum_{spikes u} Ebar_k^u.
template <typename real>
__global__ __launch_bounds__(256) void k_adjoint(DevNet<real> n) {
  const uint32_t b = blockIdx.y;
  if (b >= n.ctl[CTL_NTRIALS]) return;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n.J) return;
  const uint32_t T = n.T[b], K = n.K;
  const double beta = (double)n.beta_j[j];
  const real *fbj = n.fb + (size_t)j * K;
  const double *eb = n.ebar + (size_t)b * (n.Tcap + 2) * K;
  const real *ps = n.psi + (size_t)b * (n.Tcap + 1) * n.Jp + j;
  real *ph = n.phi + ((size_t)b * n.Jp + j) * n.Tp;
  double mu0 = 0.0, mu1 = 0.0;
  for (uint32_t t = T; t >= 1; --t) {
    double L = 0.0;
    for (uint32_t k = 0; k < K; ++k) L += (double)fbj[k] * eb[(size_t)t * K + k];
    const double p = (double)ps[(size_t)t * n.Jp];
    const double pl = p * L;
    const double m0 = pl + n.alpha_d * mu0 + p * mu1;
    const double m1 = -beta * pl + (n.rho_d - p * beta) * mu1;
    ph[t] = (real)m0;
    mu0 = m0;
    mu1 = m1;
  }
  const uint32_t c = n.spk_cnt[(size_t)b * n.NS + n.I + j];
  const uint16_t *st = n.spk_t + (size_t)b * n.spk_stride + (size_t)(n.I + j) * n.Tcap;
  real *go = n.gout_b + (size_t)b * K * n.Jp + j;
  for (uint32_t k = 0; k < K; ++k) {
    double acc = 0.0;
    for (uint32_t i = 0; i < c; ++i) acc += eb[(size_t)st[i] * K + k];
    go[(size_t)k * n.Jp] = (real)acc;
  }
}

// Event-driven synapse gradient, target-major: one wavefront per target
// neuron j, one lane per incoming synapse.  For every trial of the batch
// the lane walks the presynaptic spike-time list of its source; each
// arrival a = s + D <= T adds phi_j^a.  The per-synapse sum is Kahan-added
// into the accumulator pair (gs, gc).
template <typename real>
__global__ __launch_bounds__(256) void k_synapse(DevNet<real> n) {
  const uint32_t lane = lane_id();
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t ntr = n.ctl[CTL_NTRIALS];
  unsigned long long nev = 0;
  for (uint32_t j = wave; j < n.J; j += nwaves) {
    const uint32_t q1 = n.tm_ptr[j + 1];
    for (uint32_t q = n.tm_ptr[j] + lane; q < q1; q += 64) {
      const uint32_t pk = n.tm_syn[q];
      const uint32_t src = pk & 0xFFFFFFu, D = pk >> 24;
      real s = 0, c = 0;
      for (uint32_t b = 0; b < ntr; ++b) {
        const uint32_t T = n.T[b];
        const uint32_t cnt = n.spk_cnt[(size_t)b * n.NS + src];
        const uint16_t *st = n.spk_t + (size_t)b * n.spk_stride + (size_t)src * n.Tcap;
        const real *ph = n.phi + ((size_t)b * n.Jp + j) * n.Tp;
        for (uint32_t k = 0; k < cnt; ++k) {
          const uint32_t a = (uint32_t)st[k] + D;
          if (a > T) break;
          kahan_add(s, c, ph[a]);
          ++nev;
        }
      }
      real gs = n.gs[q], gc = n.gc[q];
      kahan_add(gs, gc, s);
      kahan_add(gs, gc, c);
      n.gs[q] = gs;
      n.gc[q] = gc;
    }
  }
  for (int o = 32; o > 0; o >>= 1) nev += __shfl_down(nev, o);
  if (lane == 0 && nev) atomicAdd(&n.cnt[CNT_EVENTS], nev);
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
    n.sm_w[n.tm_perm[q]] = (real)w;
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
  if (n.I > 0) k_stage_in_lists<real><<<dim3(cdiv(n.I, 256), n.Bcap), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::stage_forced(const DevNet<real> &n, uint32_t ntr, uint64_t nf, hipStream_t s) {
  if (nf > 0) k_stage_forced<real><<<grid_for(nf, 256), 256, 0, s>>>(n, ntr, nf);
}

template <typename real>
void Launch<real>::neuron(const DevNet<real> &n, uint32_t off, bool gather, bool forced, hipStream_t s) {
  const dim3 grid(cdiv(n.Jp, 256), n.Bcap);
  if (gather) {
    if (forced) k_neuron<real, true, true><<<grid, 256, 0, s>>>(n, off);
    else k_neuron<real, true, false><<<grid, 256, 0, s>>>(n, off);
  } else {
    if (forced) k_neuron<real, false, true><<<grid, 256, 0, s>>>(n, off);
    else k_neuron<real, false, false><<<grid, 256, 0, s>>>(n, off);
  }
}

template <typename real>
void Launch<real>::deliver(const DevNet<real> &n, const Shapes &sh, uint32_t off, hipStream_t s) {
  // the input-source pointer is read from device memory so that captured
  // graphs stay valid when a batch brings new device arrays
  k_deliver<real><<<dim3(sh.deliver_blocks_per_trial, n.Bcap), sh.block, 0, s>>>(
      n, off, reinterpret_cast<const uint32_t *const *>(n.ctl + CTL_WORDS));
}

template <typename real>
void Launch<real>::readout(const DevNet<real> &n, hipStream_t s) {
  k_readout_sums<real><<<dim3(cdiv(n.Tcap, 4), n.Bcap), 256, 0, s>>>(n);
  k_readout_scan<real><<<n.Bcap, 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::adjoint(const DevNet<real> &n, hipStream_t s) {
  k_adjoint<real><<<dim3(cdiv(n.J, 256), n.Bcap), 256, 0, s>>>(n);
}

template <typename real>
void Launch<real>::synapse(const DevNet<real> &n, const Shapes &sh, hipStream_t s) {
  k_synapse<real><<<sh.syn_blocks, sh.block, 0, s>>>(n);
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

void launch_advance(uint32_t *ctl, uint32_t by, hipStream_t s) { k_advance<<<1, 64, 0, s>>>(ctl, by); }

template struct Launch<float>;
template struct Launch<double>;

}  // namespace eprop
