/* eprop.h -- C ABI of the MI355X event-driven e-prop library (libeprop_hip.so).
 *
 * The library trains recurrent spiking networks with e-prop, the online
 * approximation of the loss gradient dL/dW_ji ~ sum_t L_j^t F_kappa(e_ji^t)
 * (paper, Methods "Gradients", eq. final-gradient and eq.
 * filtered-eligibility-trace), evaluated event-driven: a synapse's gradient
 * is formed only at the arrivals of its presynaptic spikes, from the
 * archived history of its postsynaptic neuron (Results, "Event-driven weight
 * updates in e-prop"; Supplementary "Algorithms").  Weights stay fixed
 * within an iteration; gradients are summed over the samples of the
 * iteration and applied once, averaged, by gradient descent or Adam
 * (Methods "Optimization").
 *
 * Model (Methods "Neuron models", "Loss function"):
 *   a_j^t = rho a_j^{t-1} + z_j^{t-1}                 (ALIF; beta_a = 0 gives LIF)
 *   A_j^t = v_th + beta_a a_j^t
 *   v_j^t = alpha v_j^{t-1} + I_j^t - z_j^{t-1} A_j^t  (reset by subtraction)
 *   z_j^t = [v_j^t >= A_j^t and not refractory]
 *   psi_j^t = surrogate(v_j^t - A_j^t), 0 while refractory
 *   y_k^t = kappa y_k^{t-1} + sum_j W^out_kj z_j^t
 *   E_k^t = window^t * dL/dy_k^t  (MSE: y - y*; softmax cross-entropy: pi - pi*)
 *   L_j^t = sum_k B_jk E_k^t
 * with alpha = exp(-dt/tau_m), rho = exp(-dt/tau_a), kappa = exp(-dt/tau_out).
 * Time steps are t = 1..T with zero state at t = 0.  Refractoriness lasts
 * n_ref = round(t_ref/dt) steps after a spike.  Every presynaptic source
 * (input channel or recurrent neuron) emits spikes at integer steps; a
 * synapse with delay D >= 1 receives a spike emitted at step s at step
 * s + D.  I_j^t sums the weights of the synapses receiving a spike at t.
 *
 * Threading: one handle must not be used by two threads at once; separate
 * handles are independent.  Every call is synchronous with respect to the
 * host: when it returns, its results are in the caller's buffers.  All
 * device work is issued on the HIP stream given to eprop_create_network.
 *
 * Errors: every call returns an eprop_status; nothing throws across the
 * ABI.  Arguments are validated before any device work; on
 * EPROP_ERR_INVALID_ARGUMENT, EPROP_ERR_CAPACITY or EPROP_ERR_STATE the
 * handle is unchanged.  After EPROP_ERR_DEVICE or EPROP_ERR_NUMERIC the
 * handle is failed: only eprop_read_state, eprop_last_error and
 * eprop_destroy_network remain usable.  A host allocation or thread start
 * that fails inside a call returns EPROP_ERR_OUT_OF_MEMORY; inside
 * eprop_simulate_batch or eprop_apply_updates it also fails the handle.
 * eprop_last_error gives the message of the last failure on a handle.
 */
#ifndef EPROP_H
#define EPROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPROP_ABI_VERSION 4u

typedef struct eprop_network eprop_network;   /* opaque, owned by the library */

typedef enum {
  EPROP_OK = 0,
  EPROP_ERR_INVALID_ARGUMENT = -1,
  EPROP_ERR_OUT_OF_MEMORY = -2,
  EPROP_ERR_DEVICE = -3,
  EPROP_ERR_STATE = -4,
  EPROP_ERR_CAPACITY = -5,
  EPROP_ERR_NUMERIC = -6,
  EPROP_ERR_UNSUPPORTED = -7
} eprop_status;

/* Arithmetic of membrane, traces, weights and gradients.  FP32 sums the
 * per-synapse gradients with compensated (Kahan) FP32; the loss, the
 * readout reductions and the backward filters of the learning signal are
 * FP64 in both modes. */
typedef enum { EPROP_FP32 = 0, EPROP_FP64 = 1 } eprop_precision;

/* Pseudo-derivative: eq. piecewise-linear-surrogate-gradient
 * psi = gamma max(0, 1 - beta |v - A|), or eq. exponential-surrogate-gradient
 * psi = gamma exp(-beta |v - A|). */
typedef enum { EPROP_SG_PIECEWISE_LINEAR = 0, EPROP_SG_EXPONENTIAL = 1 } eprop_surrogate;

/* eq. mean-squared-error (L = 1/2 sum_t sum_k (y - y*)^2), eq. softmax with
 * eq. cross-entropy-loss (L = -sum_t sum_k pi* log pi), or the temporal mean
 * squared error of the e-prop+ classification runs (eq. temporal-mse:
 * L = (1/K) sum_t sum_k (y - y*)^2 on the one-hot label, error signal
 * E = (2/K)(y - y*)), all gated by the learning window.  Classification
 * losses predict the arg max over k of the window's summed pi (CE) or y
 * (temporal MSE). */
typedef enum { EPROP_LOSS_MSE = 0, EPROP_LOSS_SOFTMAX_CE = 1, EPROP_LOSS_TEMPORAL_MSE = 2 } eprop_loss;

/* Membrane reset after a spike: subtract the adaptive threshold
 * (eq. lif_update), or set the membrane to v_reset as in the paper's e-prop+
 * experiments (Methods, "Neuron models"): v^t = alpha v_reset + I^t after a
 * spike.  With the full reset the eligibility's membrane component restarts
 * after each postsynaptic spike (dv^t/dv^{t-1} = alpha (1 - z^{t-1})). */
typedef enum { EPROP_RESET_SUBTRACT = 0, EPROP_RESET_TO_VALUE = 1 } eprop_reset;

/* Filter of the eligibility trace (Results, "Eligibility trace filter
 * decoupled from output time constant"): F_kappa with the readout's tau_out
 * (eq. filtered-eligibility-trace), F_kappa_e with its own tau_e, or none
 * (ebar = e).  The output-weight gradient always uses F_kappa. */
typedef enum { EPROP_ETRACE_COUPLED = 0, EPROP_ETRACE_DECOUPLED = 1, EPROP_ETRACE_NONE = 2 } eprop_etrace_filter;

/* Firing-rate regularisation: the static rate over the sample
 * (eq. loss-firing-rate-regularization, eq. firing-rate-regularization) or
 * the exponential moving average of e-prop+ (eq. ema-rate, eq. ema-gradient:
 * f^t = beta f^{t-1} + (1 - beta) z^t, beta = exp(-dt/reg_tau); loss
 * c^reg/2 sum_t sum_j (f_j^t - f*)^2; the gradient adds
 * c^reg (f_j^s - f*) G_beta(e^s) for s <= T - d). */
typedef enum { EPROP_REG_STATIC = 0, EPROP_REG_MOVING_AVERAGE = 1 } eprop_reg_mode;

/* eq. gradient-descent, or Adam in the TensorFlow ordering
 * (eq. eta-adam-fast, eq. delta-w-adam-fast) with one step per iteration. */
typedef enum { EPROP_OPT_GD = 0, EPROP_OPT_ADAM = 1 } eprop_optimizer;

/* Spike delivery.  SCATTER: one wavefront per spiking source adds its
 * weights into per-target delay ring buffers with atomics (order of the
 * additions not fixed).  GATHER: every target sums its incoming synapses
 * that receive a spike, in ascending source order, inputs first
 * (deterministic, bitwise reproducible).  AUTO: GATHER for FP64, SCATTER
 * for FP32. */
typedef enum { EPROP_DELIVERY_AUTO = 0, EPROP_DELIVERY_SCATTER = 1, EPROP_DELIVERY_GATHER = 2 } eprop_delivery;

/* eprop_config.flags */
#define EPROP_FLAG_NO_GRAPH (1u << 0)   /* launch the step loop kernel by kernel, no captured HIP graph */
#define EPROP_DETERMINISTIC (1u << 1)   /* bit-reproducible results: FP64 then delivers by gather (FP32
                                           delivery is deterministic in either mode) */
#define EPROP_SHARED_WEIGHTS (1u << 2)  /* all trials of a batch use the same weights (always the case;
                                           accepted for clarity) */
#define EPROP_AUTOTUNE (1u << 3)        /* the first training batch times the candidate launch shapes
                                           (delivery variant and steps per forward launch, adjoint and
                                           synapse block sizes, the synapse kernel's prefetch of spike
                                           records and synapses per thread at a time) on the batch
                                           itself and keeps the
                                           fastest; results do not depend on the choice */
/* The two forms of scatter delivery (FP32).  LOOKUP: every tile looks up,
 * for each source that spiked in the step, the source's synapses into the
 * tile.  QUEUES: the tile that owns a spiking neuron copies the neuron's
 * synapses into one queue per target tile, and each tile then reads only
 * its own queues (device memory: max_trials x 2 x recurrent synapses x 8
 * bytes, plus small tables).  By default the queues are built where
 * recurrent rows are sparse across tiles (fewer than 4 synapses per
 * source and tile on average) and fit in a quarter of the free device
 * memory, and the autotuner may then pick either form; the flags force
 * one (QUEUES: EPROP_ERR_CAPACITY if it does not fit; FP32 scatter with
 * more than one tile per trial only, else EPROP_ERR_UNSUPPORTED). */
#define EPROP_SCATTER_LOOKUP (1u << 4)
#define EPROP_SCATTER_QUEUES (1u << 5)

/* Optional device allocator, e.g. a framework's caching allocator: every
 * device buffer of the handle is taken from dev_alloc (bytes, ctx) and
 * returned through dev_free (ptr, ctx) by eprop_destroy_network.  Buffers
 * are at least 256-byte aligned.  NULL dev_alloc = hipMalloc/hipFree. */
typedef void *(*eprop_dev_alloc_fn)(size_t bytes, void *ctx);
typedef void (*eprop_dev_free_fn)(void *ptr, void *ctx);

typedef struct {
  uint32_t abi_version;          /* EPROP_ABI_VERSION */
  int32_t precision;             /* eprop_precision */
  uint32_t n_in, n_rec, n_out;   /* I input channels, J recurrent neurons, K readouts */
  const uint8_t *is_alif;        /* [n_rec] host, 1 = adaptive threshold; NULL = all LIF; copied */
  double dt, tau_m, tau_out, v_th, t_ref, tau_a, beta_a;   /* ms; beta_a applies to ALIF neurons */
  int32_t surrogate;             /* eprop_surrogate */
  double sg_gamma, sg_beta;      /* surrogate height gamma and width factor beta */
  int32_t loss;                  /* eprop_loss */
  int32_t optimizer;             /* eprop_optimizer */
  double eta, adam_beta1, adam_beta2, adam_eps_hat;
  uint32_t max_delay;            /* largest synaptic delay in steps, 1..255 */
  uint32_t max_trials;           /* largest number of trials per eprop_simulate_batch call */
  uint32_t max_steps;            /* largest trial length T, 1..65535 */
  int32_t delivery;              /* eprop_delivery */
  uint32_t flags;                /* EPROP_FLAG_NO_GRAPH | EPROP_DETERMINISTIC | EPROP_SHARED_WEIGHTS |
                                    EPROP_AUTOTUNE | EPROP_SCATTER_LOOKUP | EPROP_SCATTER_QUEUES */
  uint32_t d_out;                /* delay d in steps of recurrent spikes to the readout, 0..65535
                                    (Supplementary, "Delay from the recurrent to the output layer":
                                    y^t integrates W_out z^{t-d}; the recurrent gradient pairs the
                                    learning signal of step t with the filtered eligibility of step
                                    t-d, the output gradient E^t with the filtered spikes of t-d) */
  uint32_t d_ls;                 /* learning-signal delay d^ls in steps, 0..65535 (Supplementary,
                                    "Generalized delays"): the recurrent and input gradients take the
                                    learning signals of steps 1+d .. T-d^ls only; the output gradient
                                    is not affected */
  uint32_t history_steps;        /* per-neuron history capacity in steps; 0 = whole trial.  The
                                    history always covers the whole trial here, so other values
                                    must be >= max_steps */
  double c_reg;                  /* static firing-rate regularisation coefficient c^reg >= 0
                                    (eq. loss-firing-rate-regularization, eq. firing-rate-
                                    regularization); 0 = off.  The rate f_j of a trial is the
                                    neuron's spike count / T (per step), the loss adds
                                    c^reg/2 sum_j (f_j - f*)^2 and the recurrent and input gradients
                                    add c^reg/T (f_j - f*) e_ji^t over steps t <= T - d */
  double f_target;               /* target rate f* in spikes per second (Hz), >= 0; the regulariser
                                    uses f_target * dt / 1000 spikes per step */
  int32_t reset_mode;            /* eprop_reset */
  double v_reset;                /* membrane after a spike with EPROP_RESET_TO_VALUE */
  int32_t etrace_filter;         /* eprop_etrace_filter */
  double tau_e;                  /* ms, > 0 with EPROP_ETRACE_DECOUPLED */
  int32_t reg_mode;              /* eprop_reg_mode */
  double reg_tau;                /* ms, > 0 with EPROP_REG_MOVING_AVERAGE */
  uint32_t isi_cutoff;           /* EPROP_BATCH_ONLINE: eprop_isi_trace_cutoff in steps (Supplementary,
                                    "History Management"): an eligibility step s counts only if
                                    s - (the synapse's last arrival at or before s) < isi_cutoff;
                                    beyond it the traces are taken as decayed.  0 = no cutoff */
  eprop_dev_alloc_fn dev_alloc;  /* NULL or the allocator above */
  eprop_dev_free_fn dev_free;    /* required with dev_alloc */
  void *alloc_ctx;
} eprop_config;

/* A projection in CSR-by-source form (host memory, copied by the call):
 * synapse q of source i (row_ptr[i] <= q < row_ptr[i+1]) targets col[q]
 * with weight w[q] and delay delay[q] in 1..max_delay (delay NULL = 1).
 * No two synapses of one projection join the same pair; the recurrent
 * projection has no self-connections.  Weights must be finite.  The order
 * of synapses given here is the order of every per-synapse array the
 * library returns. */
typedef struct {
  uint32_t n_src, n_tgt;
  uint64_t nnz;
  const uint64_t *row_ptr;   /* [n_src+1] */
  const uint32_t *col;       /* [nnz] */
  const double *w;           /* [nnz] */
  const uint8_t *delay;      /* [nnz] or NULL */
} eprop_projection;

/* Adam state to resume from (host, copied); NULL pointers = zero. */
typedef struct {
  const double *m_in, *v_in;     /* [nnz of in_rec] */
  const double *m_rec, *v_rec;   /* [nnz of rec_rec] */
  const double *m_out, *v_out;   /* [n_out*n_rec] */
  uint64_t step;                 /* Adam steps taken so far */
} eprop_optimizer_state;

/* Creates a network (Methods "Network architecture"): I inputs, J LIF/ALIF
 * recurrent neurons, K leaky readouts, weights W^in (in_rec: I -> J),
 * W^rec (rec_rec: J -> J), W^out ([K*J] row-major, row k = weights into
 * readout k) and fixed random feedback B ([J*K] row-major, row j) that
 * replaces W^out^T in the learning signal (eq. replace-wkj-by-bjk).
 * opt may be NULL.  hip_stream is a hipStream_t (NULL = default stream)
 * that stays owned by the caller and must outlive the handle.  Device
 * memory is owned by the handle until eprop_destroy_network.
 * The per-trial archives (psi, the arrival archive, spike bitsets, spike-time
 * lists and the spike table) hold whole trials: about 12 bytes per neuron
 * (input or recurrent) and step in FP32, 20 in FP64, times max_trials x
 * max_steps.
 * Errors: INVALID_ARGUMENT (bad sizes, NULL arrays, delay out of range,
 * duplicate pairs, self-connections, non-finite weights, more than 2^24-1
 * sources or targets, 2^32 or more synapses), UNSUPPORTED (ABI version),
 * CAPACITY (the archives of max_trials trials of max_steps steps exceed the
 * device's free memory), OUT_OF_MEMORY, DEVICE (no usable gfx950 device). */
eprop_status eprop_create_network(const eprop_config *cfg, const eprop_projection *in_rec,
                                  const eprop_projection *rec_rec, const double *w_out,
                                  const double *feedback, const eprop_optimizer_state *opt,
                                  void *hip_stream, eprop_network **out_net);

typedef enum { EPROP_MEM_HOST = 0, EPROP_MEM_DEVICE = 1 } eprop_memory;

/* eprop_batch.flags */
#define EPROP_BATCH_TRAIN (1u << 0)    /* accumulate e-prop gradients of these trials */
#define EPROP_TRAIN EPROP_BATCH_TRAIN
#define EPROP_BATCH_PROFILE (1u << 1)  /* time each phase with HIP events (phase_ms) */
#define EPROP_RECORD_SPIKES (1u << 2)  /* keep the batch's spikes for eprop_read_state (always kept) */
#define EPROP_RECORD_TRACES (1u << 3)  /* keep psi, y, E, L, v for eprop_read_state (always kept) */
#define EPROP_BATCH_TIME_DRIVEN (1u << 4)  /* with TRAIN: the gradient by the time-driven recursion of
                                              Alg. "time-driven gradient computation" (every synapse,
                                              every step) instead of the event-driven path; the same
                                              result, kept as the baseline the event-driven path is
                                              measured against */
#define EPROP_BATCH_ONLINE (1u << 5)  /* the e-prop+ update schedule (Results, "Weight updates with every
                                         spike", "Continuous dynamics"): the batch's trials are samples
                                         run back to back by one network instance from rest, its state
                                         carried from sample to sample; every presynaptic spike first
                                         updates its synapse's weight by gradient descent (w -= eta g)
                                         over the eligibility steps s not yet used whose learning signal
                                         L^{s+d} has reached the neuron (s <= a - 1 - d^ls - d for an
                                         arrival at step a), then is delivered with the new weight; a
                                         readout synapse does the same when its presynaptic spike reaches
                                         the readout (E^{r+d} zbar^r, r <= a - 1 - d).  Gradients the
                                         run ends before using are dropped.  Weights change during the
                                         call; nothing is accumulated for eprop_apply_updates.  Host-
                                         memory batches, gradient descent, no static rate regulariser;
                                         the samples' total length must not exceed max_steps.  The loss
                                         and prediction are reported per sample; the recordings
                                         (eprop_read_state, trial 0) cover the whole run */

/* A batch of independent trials (samples) of uneven lengths, simulated
 * together from zero state with the current weights (Results, "Evidence
 * accumulation": parallel copies equal sequential processing when state
 * and traces are reset per sample).
 *   n_steps, label:   host arrays [n_trials] (always host memory);
 *   in_ptr [n_trials+1], in_step, in_src: the input spikes of trial b are
 *       entries in_ptr[b] .. in_ptr[b+1]-1, emission steps in [0, T_b-1],
 *       sorted by (step, source) within the trial; n_in_spikes = in_ptr[n_trials];
 *   target [n_trials * step_stride * n_out]: MSE target, entry
 *       ((b*step_stride) + t-1)*n_out + k is y*_k at step t;
 *   window [n_trials * step_stride] or NULL (always open): 1 where the
 *       learning window is open at step t (entry b*step_stride + t-1);
 *   forced_*: teacher forcing, NULL = free running; otherwise the recurrent
 *       spikes of trial b are exactly the (step, neuron) pairs
 *       forced_ptr[b] .. forced_ptr[b+1]-1 with steps in [1, T_b];
 *   memory: where in_ptr, in_step, in_src, target, window and forced_* live.
 *       With EPROP_MEM_DEVICE they are read by kernels, which check ranges
 *       and order and make the call fail with INVALID_ARGUMENT. */
typedef struct {
  uint32_t n_trials;
  int32_t memory;                 /* eprop_memory */
  const uint32_t *n_steps;
  uint64_t n_in_spikes;
  const uint64_t *in_ptr;
  const uint32_t *in_step, *in_src;
  uint32_t step_stride;           /* >= max n_steps */
  const double *target;           /* MSE only */
  const uint32_t *label;          /* cross-entropy only, < n_out */
  const uint8_t *window;
  uint64_t n_forced;
  const uint64_t *forced_ptr;
  const uint32_t *forced_step, *forced_neuron;
  uint32_t flags;                 /* EPROP_BATCH_* */
} eprop_batch;

#define EPROP_N_PHASES 8
/* phase_ms indices */
#define EPROP_PHASE_STAGE 0      /* input staging */
#define EPROP_PHASE_FORWARD 1    /* neuron updates and spike delivery, all steps */
#define EPROP_PHASE_READOUT 2    /* readout, error signals, loss */
#define EPROP_PHASE_ADJOINT 3    /* per-neuron archive of arrival values */
#define EPROP_PHASE_SYNAPSE 4    /* event-driven synapse gradient */
#define EPROP_PHASE_OUTPUT 5     /* output-synapse gradient reduction */

typedef struct {
  double *loss;                  /* [n_trials] caller-owned or NULL: per-trial loss */
  uint32_t *predicted;           /* [n_trials] or NULL: argmax_k of the window-summed pi (CE) */
  uint64_t n_rec_spikes, n_in_spikes;
  uint64_t n_syn_events;         /* input + recurrent deliveries arriving within their trial (TRAIN) */
  uint64_t n_out_events;         /* recurrent spikes x readouts */
  uint64_t n_eprop_updates;      /* arrival evaluations on plastic synapses (TRAIN only) */
  uint64_t n_flush_updates;      /* trial-end evaluations: (synapse, trial) pairs with at least one
                                    arrival (TRAIN only) */
  double device_seconds;         /* device time of the whole call (HIP events) */
  double phase_ms[EPROP_N_PHASES];   /* with EPROP_BATCH_PROFILE */
} eprop_batch_result;

/* Simulates the batch and, with EPROP_BATCH_TRAIN, adds the e-prop gradient
 * of every trial to the handle's accumulators (Results, "Event-driven
 * weight updates in e-prop": gradients accumulated per sample, weights
 * unchanged until eprop_apply_updates).  res is caller-owned.
 * Errors: INVALID_ARGUMENT, CAPACITY (n_trials > max_trials or a trial
 * longer than max_steps), STATE (failed handle), DEVICE, NUMERIC (a
 * non-finite loss). */
eprop_status eprop_simulate_batch(eprop_network *net, const eprop_batch *batch,
                                  eprop_batch_result *res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * as eprop_simulate_batch, with the same results, but the call allocates
 * nothing.  Host-memory batch arrays (in_step, in_src, target, window,
 * forced_step, forced_neuron) are copied into a static device array of
 * EPROP_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends, instead of into staging buffers the handle grows; the
 * step loop runs kernel by kernel where its HIP graph has not been built by
 * an earlier eprop_simulate_batch; a pending EPROP_AUTOTUNE waits for the
 * next eprop_simulate_batch.  Every call on one GPU, from any handle, shares
 * that GPU's array, so calls that overlap on one GPU race.
 * Errors: as eprop_simulate_batch; CAPACITY also when the batch's host arrays
 * (each rounded up to 256 bytes) exceed EPROP_NOALLOC_SCRATCH_BYTES;
 * UNSUPPORTED with EPROP_BATCH_ONLINE or EPROP_BATCH_TIME_DRIVEN. */
#define EPROP_NOALLOC_SCRATCH_BYTES (64u << 20)
eprop_status eprop_simulate_batch_noalloc(eprop_network *net, const eprop_batch *batch,
                                          eprop_batch_result *res);

/* Ends an iteration: divides the accumulated gradients by the number of
 * trials trained since the last call (reading: mean over the mini-batch),
 * applies gradient descent or one Adam step to W^in, W^rec and W^out, and
 * clears the accumulators (Methods "Optimization").
 * Errors: STATE (no trials trained since the last call, or failed handle),
 * DEVICE. */
eprop_status eprop_apply_updates(eprop_network *net);

typedef enum {
  EPROP_STATE_W_IN = 0,      /* double [nnz_in], caller's synapse order */
  EPROP_STATE_W_REC = 1,     /* double [nnz_rec] */
  EPROP_STATE_W_OUT = 2,     /* double [K*J] */
  EPROP_STATE_GRAD_IN = 3,   /* double, accumulated gradient sums (not yet averaged) of the
                                trials trained since the last eprop_apply_updates (zeros if none) */
  EPROP_STATE_GRAD_REC = 4,
  EPROP_STATE_GRAD_OUT = 5,
  EPROP_STATE_ADAM_M_IN = 6, EPROP_STATE_ADAM_V_IN = 7,
  EPROP_STATE_ADAM_M_REC = 8, EPROP_STATE_ADAM_V_REC = 9,
  EPROP_STATE_ADAM_M_OUT = 10, EPROP_STATE_ADAM_V_OUT = 11,
  EPROP_STATE_ADAM_STEP = 12,  /* uint64 */
  EPROP_STATE_SPIKES = 13,     /* last batch, trial `trial`: uint32 pairs (step, neuron), sorted */
  EPROP_STATE_PSI = 14,        /* last batch, trial: double [T_b * J], row t-1 */
  EPROP_STATE_Y = 15,          /* last batch, trial: double [T_b * K] readout signal */
  EPROP_STATE_ERR = 16,        /* last batch, trial: double [T_b * K] error signal E */
  EPROP_STATE_V = 17,          /* last batch, trial: double [J] membrane potential at T_b */
  EPROP_STATE_LAYOUT = 18,     /* uint64 [18]: neurons per tile, tiles per trial, bytes per
                                  delay-ring entry (4: 32-bit fixed point in FP32, 8: double in
                                  FP64), threads per tile,
                                  synapse-kernel threads, trials per synapse block, steps per
                                  forward launch, gather delivery (0/1), synapses per delivery
                                  piece, pieces in flight per lane group, adjoint-kernel
                                  threads, autotuned (0/1), entries of a tile's delivery piece
                                  table, spike-index blocks the synapse kernel loads with a
                                  record's header, synapses a synapse-kernel thread takes at
                                  a time, weight update by tile blocks (1) or in target-major
                                  order (0), trials per launch of the tiled forward kernel
                                  (as many as the device keeps resident together), scatter
                                  delivery through per-tile queues (1) or by lookup (0) */
  EPROP_STATE_L = 19,          /* last batch, trial: double [T_b * J] learning signal
                                  L_j^t = sum_k B_jk E_k^t (eq. final-gradient), row t-1 */
  EPROP_STATE_INPUT_BOUND = 20 /* double [1]: the bound on |input current| of one step used to
                                  size the FP32 fixed-point delay ring: the largest sum of |w|
                                  over one target's incoming synapses, with a small margin
                                  (recomputed by create and by every update) */
} eprop_state_id;

/* Copies one state array to host memory dst (dst_bytes large).  With
 * dst == NULL only *bytes_needed is set.  trial selects the trial of the
 * last simulated batch for per-trial states and is ignored otherwise.
 * Errors: INVALID_ARGUMENT (unknown id, trial out of range, dst too small),
 * STATE (per-trial state requested before any batch), DEVICE. */
eprop_status eprop_read_state(const eprop_network *net, int32_t what, uint32_t trial, void *dst,
                              size_t dst_bytes, size_t *bytes_needed);

/* Releases the handle and its device memory.  NULL is allowed. */
void eprop_destroy_network(eprop_network *net);

/* Static text for a status code. */
const char *eprop_status_string(int32_t status);

/* Message of the last failure on this handle ("" if none); valid until the
 * next call on the handle.  NULL handle: the last failure of
 * eprop_create_network in this thread. */
const char *eprop_last_error(const eprop_network *net);

#ifdef __cplusplus
}
#endif
#endif /* EPROP_H */
