/* CPU reference for event-driven e-prop: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, FP64 implementation of what the GPU library computes,
 * written from the paper's equations (Methods: neuron models, loss
 * function, gradients, optimization) and its algorithms (Alg. "time-driven
 * gradient computation"; Algs. "event-driven weight update" with a FIFO of
 * presynaptic spikes and its optimized spike-time form).  It shares no code,
 * header, table or helper with the HIP library; only tests, the smoke check
 * and the benchmark's CPU-baseline leg may call it.
 *
 * Conventions: steps t = 1..T, state zero at t = 0; a spike emitted by a
 * source at step s reaches a synapse with delay D at step s + D; input
 * emission steps lie in [0, T-1]; projections are CSR by source.
 */
#ifndef EPROP_ORACLE_H
#define EPROP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_src, n_tgt;
  long nnz;
  const unsigned long *row_ptr;   /* [n_src+1] */
  const unsigned int *col;        /* [nnz] target index */
  const double *w;                /* [nnz] */
  const unsigned char *delay;     /* [nnz], >= 1 */
} orc_proj;

typedef struct {
  int n_in, n_rec, n_out;
  const unsigned char *is_alif;   /* [n_rec] */
  double dt, tau_m, tau_out, v_th, t_ref, tau_a, beta_a;
  int surrogate;                  /* 0 piecewise linear, 1 exponential */
  double sg_gamma, sg_beta;
  int loss;                       /* 0 mean squared error, 1 softmax cross-entropy, 2 temporal mean
                                     squared error on the one-hot label (eq. temporal-mse) */
  orc_proj in, rec;
  const double *w_out;            /* [K*J], row k */
  const double *fb;               /* [J*K], row j */
  /* generalised delays (Supplementary, "Generalized delays") and static
   * firing-rate regularisation (Methods, "Firing rate regularization") */
  int d_out;                      /* delay d from the recurrent to the output layer, >= 0 */
  int d_ls;                       /* delay d^ls of the learning signal, >= 0 */
  double c_reg;                   /* regularisation strength c^reg (0 = off) */
  double f_target;                /* target rate f^*, in spikes per step */
  /* e-prop+ components (Results, "Event-driven e-prop with additional
   * biological features") */
  int reset_mode;                 /* 0: subtract the threshold (eq. lif_update); 1: reset to v_reset */
  double v_reset;
  int etrace_filter;              /* eligibility filter: 0 F_kappa (tau_out), 1 F_kappa_e (tau_e), 2 none */
  double tau_e;
  int reg_mode;                   /* 0 static rate (eq. loss-firing-rate-regularization), 1 exponential
                                     moving average (eq. ema-rate, eq. ema-gradient) */
  double reg_tau;                 /* the moving average's time constant: beta = exp(-dt/reg_tau) */
} orc_net;

typedef struct {
  int n_steps;
  long n_in_spikes;
  const unsigned int *in_step, *in_src;   /* emission steps in [0, T-1] */
  const double *target;                   /* [T*K] (MSE) or NULL */
  int label;                              /* class (cross-entropy, temporal MSE) */
  const unsigned char *window;            /* [T] learning window, NULL = always open */
  int forced;                             /* 1: recurrent spikes replaced by the list below */
  long n_forced;
  const unsigned int *forced_step, *forced_neuron;   /* steps in [1, T] */
} orc_trial;

typedef struct {       /* optional per-step recordings, row t-1; any may be NULL */
  double *v, *a, *psi, *learn;    /* [T*J] */
  double *y, *err;                /* [T*K] */
  unsigned char *z;               /* [T*J] */
} orc_trace;

/* One trial from zero state.  grad_mode 0: dynamics and loss only;
 * 1: time-driven gradient (per-step recursion for every synapse);
 * 2: event-driven gradient (intervals between presynaptic arrivals, walked
 * from archived postsynaptic history when the next arrival comes, flushed at
 * the end of the trial).  Gradients are ADDED into g_in [nnz_in],
 * g_rec [nnz_rec] and g_out [K*J].  *pred (classification losses) is the
 * arg max over the readouts of the learning window's summed softmax output
 * (cross-entropy) or readout signal (temporal MSE), lowest index on ties;
 * 0 for MSE.  Returns 0, or -1 on bad input. */
int orc_run_trial(const orc_net *net, const orc_trial *trial, int grad_mode,
                  double *g_in, double *g_rec, double *g_out,
                  orc_trace *trace, double *loss, int *pred);

/* e-prop gradient by forward-mode dual numbers on the neuron equations
 * (surrogate derivative for the spike, stop-gradient on the reset term and
 * on presynaptic spikes), combined with the learning signal in its
 * future-sum form.  O(T^2) per weight; tiny networks only.  Writes g_in,
 * g_rec (not accumulated). */
int orc_bruteforce_eprop(const orc_net *net, const orc_trial *trial,
                         double *g_in, double *g_rec);

/* Forward-mode gradient of the loss through the whole network (no
 * stop-gradient on presynaptic spikes; reset term still stopped; loss
 * tangent through the readouts with W_out).  Tiny networks only. */
int orc_forward_mode_loss_grad(const orc_net *net, const orc_trial *trial,
                               double *g_in, double *g_rec);

/* Teacher-forced trial: computes the loss from the forced spikes of all
 * neurons, and for each sampled target neuron its surrogate-gradient trace
 * psi_out [n_sample*T] and the time-driven gradient of each of its incoming
 * synapses (written into g_in / g_rec at the synapse's index; other entries
 * untouched).  Cost is linear in the sampled neurons' in-degrees. */
int orc_forced_sampled(const orc_net *net, const orc_trial *trial, int n_sample,
                       const int *targets, double *g_in, double *g_rec,
                       double *psi_out, double *loss);

/* What checking an FP32 evaluation of teacher-forced trial `trial` needs,
 * from running error analysis (Wilkinson; Higham, Accuracy and Stability of
 * Numerical Algorithms, sec. 3.3), to first order in u = 2^-24:
 *   psi_own, psi_bound [n_t * T] (row n = the n-th target, column t-1): the
 *     surrogate gradient psi of the forced trial (FP64) and a bound of the
 *     error of its FP32 evaluation: weights are FP32 numbers (the same on
 *     both sides); the input current of a step is the exact sum of the
 *     arriving weights rounded once to FP32, plus at most `quantum` per
 *     arriving weight (0 for an exact sum); the neuron recursion
 *     (eq. spike-threshold-adaptation, adaptive threshold, eq. lif_update,
 *     the surrogate) runs in FP32 in the order of its definition with one
 *     rounding per operation, alpha, rho, v_th, gamma and beta rounded to FP32
 *     and exp within 2 ulp;
 *   g_in, g_rec: the gradient of Alg. "time-driven gradient computation"
 *     evaluated on the archived psi history psi_given ([n_t * T], laid out
 *     like psi_own; NULL = the trial's own psi), as orc_forced_sampled;
 *     g_out [K*J] the
 *     output gradient (eq. eprop-output-new-subs-rewritten);
 *   b_in, b_rec, b_out: 7 u times the sum of the absolute values of the terms
 *     of each of these gradients (for the input and recurrent synapses,
 *     sum_t sum_k |B_jk E_k^{t+d}| times the eligibility recursion run on
 *     absolute values, plus the regularisers' terms likewise), a bound of the
 *     rounding of an FP32 evaluation downstream of psi: 1 u feedback weights
 *     rounded to FP32, 1 u stored archive values, 2 u compensated summation
 *     per synapse, 1 u stored partial sums, 2 u compensated summation of the
 *     partials.
 * Spikes (forced) and refractory states are the same on both sides.
 * n_sample < 0: every neuron is a target (n_t = J); otherwise only the
 * listed targets (n_t = n_sample) get psi rows and their incoming synapses
 * get values in g_* / b_* (written at the synapse's index, other entries
 * untouched).  Any output pointer may be NULL.  Returns 0, or -1 on bad
 * input or a trial without forced spikes. */
int orc_fp32_bounds(const orc_net *net, const orc_trial *trial, double quantum, const double *psi_given,
                    int n_sample, const int *targets, double *psi_own, double *psi_bound, double *g_in,
                    double *g_rec, double *g_out, double *b_in, double *b_rec, double *b_out);

/* e-prop+ update schedule (Results, "Weight updates with every spike";
 * Alg. "event-driven weight update" applied at every spike): one network
 * instance runs through n_samples samples back to back, its state (neurons,
 * readout, synaptic traces, histories) carried from one to the next
 * (Results, "Continuous dynamics").  A spike arriving at a synapse at step a
 * first updates the synapse's weight by gradient descent, w -= eta g, with
 * g the e-prop gradient over the eligibility steps s not yet used whose
 * learning signal L^{s+d} has reached the neuron, s <= a - 1 - d^ls - d
 * (plus the moving-average regulariser's c (f^s - f*) G_beta(e^s)); the
 * spike is then transmitted with the new weight.  A readout synapse j -> k
 * does the same when z_j arrives at the readout, with E_k^{r+d} zbar_j^r over
 * r <= a - 1 - d.  With cutoff > 0 an eligibility step s contributes only if
 * s - (the synapse's last arrival at or before s) < cutoff; beyond that the
 * traces are taken as zero (eprop_isi_trace_cutoff).  Gradients the run
 * ends before using are dropped, unless flush is set, which applies them at
 * the end as if a spike arrived after the last step.
 * Weights w_in, w_rec, w_out are updated in place (the network's own weight
 * arrays are not used); g_in, g_rec, g_out, if not NULL, accumulate every
 * gradient applied; loss [n_samples] gets each sample's loss; z, if not
 * NULL, the recurrent spikes [T_total*J]; a_in, a_rec, a_out, if not NULL,
 * accumulate |eta| times the sum of the absolute values of the terms of
 * every gradient applied (each eligibility recursion also run on absolute
 * values, the learning signal as sum_k |B_jk E_k|), the scale of the
 * rounding of an FP32 evaluation of the run's updates.  Static rate
 * regularisation and Adam have no per-spike form here; returns -1 for them. */
int orc_run_online(const orc_net *net, int n_samples, const orc_trial *samples, double eta, int cutoff,
                   int flush, double *w_in, double *w_rec, double *w_out, double *g_in, double *g_rec,
                   double *g_out, double *loss, unsigned char *z, double *a_in, double *a_rec, double *a_out);

/* End of iteration: G = g_sum / n_trials, then gradient descent or Adam in
 * the TensorFlow ordering (step = iteration count, starting at 1). */
void orc_apply(long n, double *w, const double *g_sum, double n_trials, int optimizer,
               double eta, double beta1, double beta2, double eps_hat, long step,
               double *m, double *v);

#ifdef __cplusplus
}
#endif
#endif
