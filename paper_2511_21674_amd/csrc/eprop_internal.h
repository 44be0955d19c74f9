// Internal device-side description of one network and the launchers of
// its kernels.  Shared by eprop_kernels.hip and eprop_host.cpp only.
//
// HBM layout (b = trial slot, j = neuron, t = step 1..T, Jp = J padded to 64):
//   graph, source-major  sm_ptr[NS+1] (row of each source, sorted by target)
//   delivery table       (scatter delivery) dlw: the weights and ring offsets of every
//                        (source, tile) segment, source by source, tile by tile; a
//                        segment of L synapses is L weights (real) followed by L uint16
//                        ring offsets d * TS + (target - k * TS), its size rounded up to
//                        a multiple of sizeof(real); it starts on a kDlGrain-byte
//                        boundary if it would otherwise cross one it need not cross
//                        (so that a delivery reads as few lines as the segment's size
//                        allows); tiles in tile_rank order; dseg[src][tile_rank(k)] =
//                        {word index of the segment, L}
//   graph, target-major  tm_ptr[J+1], tm_syn[S] = source | delay << 24, tm_w[S]
//                        (sources: inputs 0..I-1, then recurrent I..I+J-1;
//                        each target's list sorted by source), tm_dpos[S]
//                        (target-major index -> word index of the synapse's weight in dlw)
//   gradient sums        gs[S], gc[S] (Kahan pair, target-major), Adam m, v (source-major
//                        with scatter delivery, target-major with gather delivery)
//   weight update        (scatter delivery, rows dense within a tile) blocks
//                        ach[3 * n_ach] = (tile, first source, end source), each at most
//                        kApplySyn synapses into one tile's targets; trs[n_ach][TS]: where
//                        each target's run of the block's sources starts in its row;
//                        tsum[Jp] per-target sum of |w| in fixed point (the input bound)
//   neuron state         v[b][Jp], a[b][Jp], nst[b][Jp] (refractory count | z << 7)
//   delay ring           ring[b][R][Jp], R = max_delay + 1 (scatter delivery; held in
//                        LDS by the tile that owns the targets, saved between launches;
//                        FP32: 32-bit fixed point with scale 2^-F; FP64: double)
//   input bound          l1max: max over targets of the sum of |w| of incoming
//                        synapses (FP32 bits), which fixes F
//   tile segments        tseg[src][k], k = 0..KT: first synapse of source src whose
//                        target lies in tile k (source rows sorted by target)
//   psi archive          psi[b][t][Jp]          (time-major, written per step)
//   arrival archive      phi[b][j][t]           (neuron-major, stride Tp)
//   spike bitsets        rec_bits[b][t][Jw], in_bits[b][s][Iw], forced_bits[b][t][Jw]
//   spike-time lists     spk_cnt[b][NS], spk_t[b][src*Lc + k] (uint16, ascending)
//   per-step spikes      pub_list[b][t & 1][Jp] (tile k's spiking neurons of step t at
//                        k*TS.., each word t << 32 | j), pub_cnt[b][t & 1][KT]
//                        (t << 32 | count of tile k), nspk[b][t]
//   per-tile queues      (scatter delivery through queues, FP32) q_nzp[J+1], q_nz[]: for each
//                        recurrent neuron, its non-empty tile segments {word index in dlw,
//                        L | target tile << 16}; then q_nz[q_in + i * KT + k]: input i's
//                        segment into tile (k - i) mod KT, copied by tile k;
//                        q_ev[b][t & 1][q_len]: one region per (source tile, target
//                        tile), as large as the synapses the source tile copies into the
//                        target tile, regions ordered by target tile, then source tile;
//                        q_src[k][kd]
//                        (= q_dst[kd][k]): where region (k -> kd) starts; an event is
//                        tag16 << 48 | ring offset << 32 | weight bits; q_hdr[b][t & 1][kd][k]
//                        = tag << 32 | events of step t in region (k -> kd)
//   readout (FP64)       ysum/pi[b][t][K], y[b][t][K], err[b][t][K], ebar[b][t][K], ebo[b][t][K]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eprop {

// ctl words; the 64-bit device pointer to the batch's input-source array is
// stored at word CTL_WORDS (byte offset 64)
// (CTL_TAG0: the queues' step tags of the batch are CTL_TAG0 + t, all in 1..65535)
enum : uint32_t { CTL_T0 = 0, CTL_NTRIALS = 1, CTL_ERR = 2, CTL_TAG0 = 3, CTL_WORDS = 16 };
enum : uint32_t { ERR_INPUT_RANGE = 1u, ERR_INPUT_ORDER = 2u, ERR_FORCED_RANGE = 4u, ERR_SYNC = 8u,
                  ERR_INPUT_BOUND = 16u };
enum : uint32_t { CNT_EVENTS = 0, CNT_REC_SPIKES = 1, CNT_FLUSH = 2, CNT_WORDS = 8 };
constexpr uint32_t kScanItems = 4096;        // entries per block of the spike-table scan
constexpr uint32_t kNoRecord = 0xFFFFFFFFu;  // spike-table offset of a source without spikes
constexpr uint32_t kApplySyn = 16384;        // synapses per weight-update block (at most, FP32)
constexpr uint32_t kApplySrc = 2048;         // sources per weight-update block (at most)
constexpr uint32_t kApplyMaxTile = 8192;     // tile size the blocked update supports
constexpr double kBoundScale = 65536.0;      // fixed-point scale of the per-target |w| sums
constexpr double kBoundMaxW = 4194304.0;     // |w| from which the bound saturates (2^22)
constexpr size_t kScratchBytes = (size_t)64 << 20;  // static staging array of the no-allocation batch call
constexpr int kMaxDevices = 64;

// Placement unit of the delivery table's segments (bytes): the line a
// partial read of device memory costs.
constexpr uint32_t kDlGrain = 128;

// Order of a source's tile segments in the delivery table and in dseg:
// tiles grouped by k mod kXcds, since workgroup i of a launch runs on
// accelerator die i mod kXcds and the tiles of one trial are consecutive
// workgroups, so each die's tiles read one contiguous stretch of a source's
// row (and of its segment lookups) through their shared L2.
constexpr uint32_t kXcds = 8;
__host__ __device__ inline uint32_t tile_rank(uint32_t k, uint32_t KT) {
  const uint32_t g = k % kXcds;
  uint32_t r = k / kXcds;
  for (uint32_t h = 0; h < g; ++h) r += (KT - h + kXcds - 1) / kXcds;  // tiles of group h
  return r;
}

// Element of the delay ring.  FP32: the input current of a step is summed
// in 32-bit fixed point (int32_t, F up to 30 fraction bits; each arrival's
// weight is rounded to a multiple of 2^-F, at most 2^-31 of the input bound
// off, where an FP32 running sum of the same arrivals would round each
// addition by up to 2^-24 of it); the integer sum is exact, so it does not
// depend on the order of arrival.  Integer LDS atomics are an order of
// magnitude faster than float ones on this GPU.  F follows from l1max, so no
// sum can overflow.  FP64: plain double.

template <typename real>
struct DevNet {
  // sizes
  uint32_t I, J, K, NS, Jp, Jw, Iw, R, Tcap, Tp, Bcap;
  uint32_t Ts;                  // synapse kernel's LDS row per trial: Tcap + R rounded up to 4
  uint64_t spk_stride;          // per-slot size of spk_t (NS * Lc)
  uint32_t Lc;                  // spike-list capacity per source (Tcap rounded up to 8)
  uint64_t S;                   // synapses
  uint32_t n_ref;
  int32_t surrogate, loss;
  uint32_t step_stride;         // batch target/window row length
  uint32_t TS, KT;              // tile size (neurons), tiles per trial
  uint32_t ptab_cap;            // entries of the forward tile's piece table (>= its threads)
  // constants (working precision for the dynamics, FP64 for the backward filters)
  real alpha, rho, v_th, sg_gamma, sg_beta;
  double alpha_d, rho_d, kappa_d;
  uint32_t d_out, d_ls;         // readout delay d, learning-signal delay d^ls (steps)
  double c_reg, f_target;       // rate regulariser coefficient and target rate (spikes per step)
  int32_t reset_mode;           // 0 subtract the threshold, 1 reset to v_reset
  real v_reset;
  double kappa_e_d;             // the eligibility filter's factor (kappa unless decoupled; 0: none)
  int32_t reg_mode;             // 0 static rate, 1 moving average (only with c_reg != 0)
  double beta_f;                // the moving average's factor
  // graph
  const uint32_t *sm_ptr, *tseg;
  uint32_t *dlw;                // delivery table (scatter delivery; null with gather delivery)
  const uint2 *dseg;            // [NS][KT] {word index in dlw, synapse count} of each segment
  uint32_t ts_magic;            // floor(2^32 / TS) + 1: o / TS == (o * ts_magic) >> 32 for o < 2^16
  const uint32_t *tm_ptr, *tm_syn, *tm_dpos;
  real *tm_w;                   // target-major weights (gather delivery only)
  real *gs, *gc, *adam_m, *adam_v;
  int32_t g_fresh;              // no trial accumulated since the last update: gradient kernels write gs/gc, not add
  const uint32_t *ach;          // blocked update: blocks (tile, first source, end source)
  const uint32_t *trs;          // blocked update: [n_ach][TS] start of each target's run
  const uint16_t *tm_loc;       // blocked update: [S] each synapse's place in its block's source-major segments
  unsigned long long *tsum;     // blocked update: [Jp] per-target sum of |w| * kBoundScale
  const real *beta_j;           // beta_a for ALIF neurons, 0 for LIF [Jp]
  real beta_a;                  // the ALIF neurons' beta_a
  int32_t any_alif;             // some beta_j is nonzero
  real *w_out, *fb;             // [K][Jp], [Jp][K]
  real *gos, *goc, *adam_mo, *adam_vo;   // [K][Jp]
  real *gout_b;                 // [Bcap][K][Jp]
  // per-slot state
  real *v, *a;
  uint8_t *nst;
  void *ring;                   // ring_t [Bcap][R][Jp]
  uint32_t ring_bytes;          // 4: int32_t (FP32); 8: double (FP64)
  real *psi, *phi;
  uint32_t *l1max;              // [1] bound on |input current| per step (FP32 bits)
  uint64_t *rec_bits, *in_bits, *forced_bits;
  uint32_t *spk_cnt;
  uint16_t *spk_t;
  // per-source spike table of a batch for the synapse kernel: record (c, i)
  // of trial chunk c and source i = 16-byte header of 8 uint16 spike counts,
  // then one uint16 per spike, the LDS index bi * Ts + t of spike time t of
  // the chunk's trial bi, trial by trial, padded to a multiple of 8 with the
  // index of a zero entry
  const uint32_t *outdeg;       // [NS][R] out-degree of each source per delay (index 1..R-1)
  uint32_t *pk_off;             // [nchunk*NS + 1] record offset in 16-byte units, kNoRecord if empty
  uint32_t *pk_bsum;            // [scan blocks + 1]
  uint16_t *pk;                 // [pk_cap * 8]
  uint64_t pk_cap;
  uint64_t *pub_list, *pub_cnt;
  // per-tile queues (null unless built)
  const uint32_t *q_nzp, *q_src, *q_dst;
  const uint2 *q_nz;
  uint64_t *q_ev, *q_hdr;
  uint32_t q_len;               // events per (trial, parity) buffer: the synapses
  uint32_t q_in;                // where the input entries of q_nz start
  uint32_t *nspk;
  uint64_t *in_step_ptr;        // [Bcap][Tcap+1]
  double *ysum, *y, *err;       // [Bcap][Tcap+2][K]
  double *ebar;                 // [Bcap][Tcap+2][K] backward-filtered error paired with the
                                // eligibility of step u: sum_{v=u}^{T-d-d^ls} kappa^{v-u} E^{v+d}
  double *ebo;                  // the same with the readout's kappa and without the learning-signal
                                // cut (upper end T-d), for the output gradient; aliases ebar when
                                // d^ls = 0 and the eligibility filter is the readout's
  double *loss_out;             // [Bcap]
  uint32_t *pred_out;           // [Bcap]
  // batch (device pointers)
  const uint32_t *T, *label;
  const uint64_t *in_ptr;
  const uint32_t *in_step, *in_src;
  const double *target;
  const uint8_t *window;
  const uint64_t *forced_ptr;
  const uint32_t *forced_step, *forced_neuron;
  // control
  uint32_t *ctl;
  unsigned long long *cnt;
  unsigned long long *evcnt;    // [64] event counters (spread to avoid one hot atomic)
};

// e-prop+ update schedule (weight update at every arriving spike, one
// continuous run): per-synapse state in target-major order, and the run's
// readout state and histories.
template <typename real>
struct OnlineSyn {
  real ev, ea, eb, gh;          // eligibility vector, filtered trace, G_beta-filtered trace
  uint32_t s_done;              // last eligibility step used
  uint32_t last;                // last arrival at or before s_done (0: none)
};

template <typename real>
struct OnlineRun {
  OnlineSyn<real> *syn;         // [S]
  double *Eh;                   // [T+1][K] error signals of the run
  double *y;                    // [K] readout state
  double *zbo;                  // [Jp] zbar of each neuron for its readout synapses
  uint32_t *r_done, *zlast;     // [Jp] readout synapses: last step used, last spike
  real *fh;                     // [T+1][Jp] moving-average rates (moving-average regulariser)
  real *Ibuf;                   // [Jp] input current of the step, from the synapse side
  real *Lh;                     // [T+1][Jp] learning signals of the run
  double *loss;                 // [n_samples]
  double *psum;                 // [n_samples][K] window sums for the prediction
  const uint32_t *off;          // [n_samples+1] first step - 1 of each sample
  const uint32_t *label;        // [n_samples]
  uint32_t n_samples;
  uint32_t cutoff;              // eprop_isi_trace_cutoff in steps (0: none)
  uint32_t lag;                 // 1 + d^ls + d: the learning signal of step s + d is at the neuron at s + lag
  double eta;
};

// Launch shapes (chosen on the host; the autotuner may change them)
struct Shapes {
  uint32_t block;               // threads per block for grid-stride kernels
  uint32_t tile_block;          // threads per block of the tiled forward kernel
  uint32_t syn_block;           // threads per block of the synapse kernel
  uint32_t ginst;               // trials per block of the synapse kernel
  uint32_t fwd_variant;         // delivery variant of the forward kernel (piece size, pieces in flight)
  uint32_t adj_block;           // threads per block of the adjoint kernel (64, 128 or 256)
  uint32_t syn_var;             // synapse kernel variant: header prefetch and synapses per thread at a time
  uint32_t fwd_trials;          // trials per launch of the tiled forward kernel (all of them resident together)
};
uint32_t fwd_variant_piece(uint32_t v);
uint32_t fwd_variant_unroll(uint32_t v);
uint32_t syn_variant_pre(uint32_t v);
uint32_t syn_variant_batch(uint32_t v);
constexpr uint32_t kNumSynVariants = 7;
constexpr uint32_t kNumFwdVariants = 5;
constexpr uint32_t kQueueVariant = 4;  // the forward variant that delivers through the per-tile queues

template <typename real>
struct Launch {
  static void rec_lists(const DevNet<real> &n, uint32_t n_trials, hipStream_t s);  // after a tiled forward pass
  static void stage_inputs(const DevNet<real> &n, uint32_t n_trials, uint64_t n_spikes, bool check_order,
                           hipStream_t s);
  static void stage_forced(const DevNet<real> &n, uint32_t n_trials, uint64_t n_forced, hipStream_t s);
  // deterministic per-step neuron update with gather delivery at step ctl[T0] + off
  static void neuron_gather(const DevNet<real> &n, uint32_t off, bool forced, hipStream_t s);
  // persistent tiled forward pass over steps ctl[T0]+1 .. ctl[T0]+nsteps
  static void forward_tiled(const DevNet<real> &n, uint32_t nsteps, bool forced, const Shapes &sh,
                            size_t smem, hipStream_t s);
  static size_t tile_smem(uint32_t TS, uint32_t R, uint32_t ring_bytes, uint32_t ptab_cap);
  static hipError_t allow_smem(size_t smem, uint32_t ring_bytes);
  static hipError_t resident(uint32_t block, size_t smem, uint32_t ring_bytes, int *per_cu);
  static void readout(const DevNet<real> &n, hipStream_t s);
  static void adjoint(const DevNet<real> &n, const Shapes &sh, hipStream_t s);
  static void synapse(const DevNet<real> &n, const Shapes &sh, uint32_t n_trials, real *partial, hipStream_t s);
  static void output_reduce(const DevNet<real> &n, hipStream_t s);
  static void apply(const DevNet<real> &n, uint64_t n_syn, double n_trials, int optimizer, double eta,
                    double eta_t, double b1, double b2, double eps_hat, hipStream_t s);
  // the update as a blocked transposition (n_ach blocks of one tile's targets
  // and a range of sources), which also recomputes *l1max; gs, gc cleared
  static void apply_blocked(const DevNet<real> &n, uint32_t n_ach, uint64_t n_syn, double n_trials,
                            int optimizer, double eta, double eta_t, double b1, double b2, double eps_hat,
                            hipStream_t s);
  static void input_bound_blocked(const DevNet<real> &n, uint32_t n_ach, hipStream_t s);
  static size_t apply_blocked_smem(uint32_t TS);   // static + dynamic LDS of one update block
  // the gradient of the batch by the time-driven recursion (baseline); L: [Bcap][Tcap+1][Jp]
  static void time_driven(const DevNet<real> &n, const Shapes &sh, uint32_t n_trials, real *L, real *partial,
                          hipStream_t s);
  // recomputes *l1max from the current weights (after upload and every update)
  static void input_bound(const DevNet<real> &n, hipStream_t s);
  // e-prop+ schedule: target-major weights from / to the source-major records,
  // and one step t of the continuous run (neurons with their synapse updates,
  // then readout synapses, readout, error and loss)
  static void online_fill(const DevNet<real> &n, bool to_records, hipStream_t s);
  static void online_step(const DevNet<real> &n, const OnlineRun<real> &o, uint32_t t, bool forced, hipStream_t s);
};

void launch_advance(uint32_t *ctl, uint32_t by, hipStream_t s);

// Device address of the static staging array (kScratchBytes) of the
// no-allocation batch call on `device`, which must be the current device;
// looked up once per device and kept.  nullptr and *err set on failure.
void *scratch_address(int device, hipError_t *err);

}  // namespace eprop
