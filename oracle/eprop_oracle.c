/* CPU reference for event-driven e-prop: TEST INFRASTRUCTURE ONLY.
 *
 * Plain serial FP64 C, built with -O2 -ffp-contract=off so that every
 * multiply and add rounds on its own.  Nothing here is blocked, fused or
 * reordered beyond what the paper's equations and algorithms state.
 * Equation names refer to the paper's labels (Methods and Supplementary
 * Information).  Readings of points the paper leaves open:
 *   - a spike is emitted iff v >= threshold (the Heaviside tie spikes);
 *   - refractoriness (not in the equations): after a spike at t_s the
 *     neuron cannot spike and has psi = 0 at steps t_s+1 .. t_s+n_ref, while
 *     v keeps integrating, reset included;
 *   - the reset subtracts the current adaptive threshold v_th + beta_a a^t;
 *   - psi multiplies both eligibility components, e = psi (eps_v - beta_a eps_a)
 *     (eq. filtered-eligibility-trace; the brace in eq. gradient-rec is read
 *     the same way);
 *   - the output gradient is sum_t E_k^t F_kappa(z_j^t)
 *     (eq. eprop-output-new-subs-rewritten with d = 0);
 *   - the learning window multiplies E (and so L); loss terms outside it are 0;
 *   - every synapse sees its presynaptic spike train delayed by its own
 *     delay D >= 1; inputs enter exactly like recurrent sources;
 *   - the input current sums the arriving input synapses in ascending source
 *     order, then the arriving recurrent synapses in ascending source order.
 */
#include "eprop_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int kind;      /* 0 input, 1 recurrent */
  int src;
  int delay;
  long idx;      /* index into the projection's arrays */
} in_syn;

typedef struct {
  double alpha, kappa, rho;  /* exact-integration propagators */
  double kappa_e;            /* the eligibility trace's filter (kappa unless decoupled) */
  double beta_f;             /* the rate's moving-average factor (eq. ema-rate) */
  int n_ref;
  int max_delay;
  long *in_ptr;              /* [J+1] incoming synapses per target, canonical order */
  in_syn *syn;
} prep_t;

static void prep_free(prep_t *p) {
  free(p->in_ptr);
  free(p->syn);
}

/* Propagators of eq. lif_update, eq. spike-threshold-adaptation and
 * eq. leaky_integrator: alpha = exp(-dt/tau_m), rho = exp(-dt/tau_a),
 * kappa = exp(-dt/tau_out). */
static int prep_init(const orc_net *net, prep_t *p) {
  const int J = net->n_rec;
  memset(p, 0, sizeof(*p));
  p->alpha = exp(-net->dt / net->tau_m);
  p->kappa = exp(-net->dt / net->tau_out);
  p->rho = exp(-net->dt / net->tau_a);
  /* Results, "Eligibility trace filter decoupled from output time constant":
   * F_kappa, F_kappa_e with its own time constant, or no filter */
  p->kappa_e = net->etrace_filter == 1 ? exp(-net->dt / net->tau_e) : net->etrace_filter == 2 ? 0.0 : p->kappa;
  p->beta_f = net->reg_mode == 1 ? exp(-net->dt / net->reg_tau) : 0.0;
  p->n_ref = (int)lround(net->t_ref / net->dt);
  p->in_ptr = (long *)calloc((size_t)J + 1, sizeof(long));
  long total = net->in.nnz + net->rec.nnz;
  p->syn = (in_syn *)malloc(sizeof(in_syn) * (size_t)(total > 0 ? total : 1));
  long *fill = (long *)calloc((size_t)J + 1, sizeof(long));
  if (!p->in_ptr || !p->syn || !fill) { free(fill); prep_free(p); return -1; }
  const orc_proj *pr[2] = {&net->in, &net->rec};
  for (int kind = 0; kind < 2; ++kind)
    for (long q = 0; q < pr[kind]->nnz; ++q) {
      unsigned int j = pr[kind]->col[q];
      if ((int)j >= J || pr[kind]->delay[q] < 1) { free(fill); prep_free(p); return -1; }
      p->in_ptr[j + 1]++;
      if (pr[kind]->delay[q] > p->max_delay) p->max_delay = pr[kind]->delay[q];
    }
  for (int j = 0; j < J; ++j) p->in_ptr[j + 1] += p->in_ptr[j];
  /* sources visited in ascending order, inputs first: lists come out canonical */
  for (int kind = 0; kind < 2; ++kind)
    for (int i = 0; i < pr[kind]->n_src; ++i)
      for (unsigned long q = pr[kind]->row_ptr[i]; q < pr[kind]->row_ptr[i + 1]; ++q) {
        unsigned int j = pr[kind]->col[q];
        in_syn *s = &p->syn[p->in_ptr[j] + fill[j]++];
        s->kind = kind;
        s->src = i;
        s->delay = pr[kind]->delay[q];
        s->idx = (long)q;
      }
  free(fill);
  return 0;
}

/* Spike records: zin[s*I + i] for emission steps s in [0, T-1];
 * zrec[t*J + j] for t in [0, T] with row 0 all zero. */
typedef struct {
  int T, I, J;
  unsigned char *zin, *zrec, *zforced;
  int *list;     /* [J] work space: the spiking neurons of one step, ascending */
} spikes_t;

static int spiked(const spikes_t *sp, int kind, int src, int s) {
  if (kind == 0) return (s >= 0 && s < sp->T) ? sp->zin[(long)s * sp->I + src] : 0;
  return (s >= 1 && s <= sp->T) ? sp->zrec[(long)s * sp->J + src] : 0;
}

static void spikes_free(spikes_t *sp) {
  free(sp->zin);
  free(sp->zrec);
  free(sp->zforced);
  free(sp->list);
}

static int spikes_init(const orc_net *net, const orc_trial *tr, spikes_t *sp) {
  memset(sp, 0, sizeof(*sp));
  sp->T = tr->n_steps;
  sp->I = net->n_in;
  sp->J = net->n_rec;
  sp->zin = (unsigned char *)calloc((size_t)sp->T * (sp->I > 0 ? sp->I : 1), 1);
  sp->zrec = (unsigned char *)calloc((size_t)(sp->T + 1) * sp->J, 1);
  sp->list = (int *)calloc((size_t)sp->J, sizeof(int));
  if (!sp->zin || !sp->zrec || !sp->list) { spikes_free(sp); return -1; }
  for (long e = 0; e < tr->n_in_spikes; ++e) {
    unsigned int s = tr->in_step[e], i = tr->in_src[e];
    if ((int)s >= sp->T || (int)i >= sp->I) { spikes_free(sp); return -1; }
    sp->zin[(long)s * sp->I + i] = 1;
  }
  if (tr->forced) {
    sp->zforced = (unsigned char *)calloc((size_t)(sp->T + 1) * sp->J, 1);
    if (!sp->zforced) { spikes_free(sp); return -1; }
    for (long e = 0; e < tr->n_forced; ++e) {
      unsigned int t = tr->forced_step[e], j = tr->forced_neuron[e];
      if (t < 1 || (int)t > sp->T || (int)j >= sp->J) { spikes_free(sp); return -1; }
      sp->zforced[(long)t * sp->J + j] = 1;
    }
  }
  return 0;
}

/* Surrogate gradient: eq. piecewise-linear-surrogate-gradient or
 * eq. exponential-surrogate-gradient, of the distance to the threshold. */
static double surrogate(const orc_net *net, double dv) {
  if (net->surrogate == 1) return net->sg_gamma * exp(-net->sg_beta * fabs(dv));
  return net->sg_gamma * fmax(0.0, 1.0 - net->sg_beta * fabs(dv));
}

static double neuron_beta(const orc_net *net, int j) {
  return (net->is_alif && net->is_alif[j]) ? net->beta_a : 0.0;
}

/* Input current of neuron j at step t: eq. lif_update's two sums, each
 * synapse seeing its source delayed by its own delay. */
static double input_current(const orc_net *net, const prep_t *p, const spikes_t *sp, int j, int t) {
  double I = 0.0;
  for (long q = p->in_ptr[j]; q < p->in_ptr[j + 1]; ++q) {
    const in_syn *s = &p->syn[q];
    if (spiked(sp, s->kind, s->src, t - s->delay))
      I = I + (s->kind == 0 ? net->in.w[s->idx] : net->rec.w[s->idx]);
  }
  return I;
}

/* One neuron update at step t (eq. spike-threshold-adaptation, adaptive
 * threshold, eq. lif_update, eq. binary-spike-state-variable, surrogate).
 * With the full reset of the e-prop+ experiments the membrane restarts
 * from v_reset after a spike instead of losing the threshold. */
static int neuron_step(const orc_net *net, const prep_t *p, int j, double I, double zprev,
                       int forced_z, double *v, double *a, int *refr, double *psi) {
  const double beta = neuron_beta(net, j);
  *a = p->rho * *a + zprev;
  const double A = net->v_th + beta * *a;
  if (net->reset_mode == 1) *v = p->alpha * (zprev != 0.0 ? net->v_reset : *v) + I;
  else *v = p->alpha * *v + I - zprev * A;
  const int refractory = *refr > 0;
  if (refractory) *refr -= 1;
  int z;
  if (forced_z >= 0) z = forced_z;
  else z = (!refractory && *v >= A) ? 1 : 0;
  *psi = refractory ? 0.0 : surrogate(net, *v - A);
  if (z) *refr = p->n_ref;
  return z;
}

/* One step of a synapse's eligibility (eq. eligibility-vector-substituted,
 * eq. filtered-eligibility-trace):
 *   eps_a^t = psi^{t-1} eps_v^{t-1} + (rho - psi^{t-1} beta) eps_a^{t-1}
 *   eps_v^t = alpha eps_v^{t-1} + x^t                   (F_alpha of the arrivals)
 *   e^t     = psi^t (eps_v^t - beta eps_a^t)
 *   ebar^t  = kappa_e ebar^{t-1} + e^t                  (F_kappa, or the decoupled filter)
 * With the full reset, dv^t/dv^{t-1} = alpha (1 - z_j^{t-1}), so eps_v
 * restarts after each postsynaptic spike (zprev = z_j^{t-1}).
 * Returns e^t; the caller pairs ebar^t with the learning signal. */
static double syn_trace(const orc_net *net, const prep_t *p, double x, double zprev, double psi_prev, double psi_now,
                        double beta, double *ev, double *ea, double *eb) {
  const double ea_new = psi_prev * *ev + (p->rho - psi_prev * beta) * *ea;
  const double ev_new = (net->reset_mode == 1 && zprev != 0.0 ? 0.0 : p->alpha) * *ev + x;
  const double e = psi_now * (ev_new - beta * ea_new);
  *eb = p->kappa_e * *eb + e;
  *ev = ev_new;
  *ea = ea_new;
  return e;
}

/* Readout (eq. leaky_integrator), error signal and loss (eq. mean-squared-error
 * or eq. softmax + eq. cross-entropy-loss), window-gated. */
static void readout_core(const orc_net *net, const prep_t *p, spikes_t *sp, int t, const double *target_row,
                         int win, int label, double *y, double *E, double *loss, double *psum);

static void readout_step(const orc_net *net, const prep_t *p, spikes_t *sp,
                         const orc_trial *tr, int t, double *y, double *E, double *loss,
                         double *psum) {
  readout_core(net, p, sp, t, tr->target ? tr->target + (long)(t - 1) * net->n_out : NULL,
               tr->window ? tr->window[t - 1] : 1, tr->label, y, E, loss, psum);
}

static void readout_core(const orc_net *net, const prep_t *p, spikes_t *sp, int t, const double *target_row,
                         int win, int label, double *y, double *E, double *loss, double *psum) {
  const int J = net->n_rec, K = net->n_out;
  /* the neurons whose spike reaches the readout now, ascending: each
   * readout sums their weights in that order */
  int n = 0;
  if (t - net->d_out >= 1)
    for (int j = 0; j < J; ++j)
      if (sp->zrec[(long)(t - net->d_out) * J + j]) sp->list[n++] = j;
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = s + net->w_out[(long)k * J + sp->list[i]];
    y[k] = p->kappa * y[k] + s;
  }
  if (net->loss == 2) {
    /* eq. temporal-mse on the one-hot label: L = (1/K) sum_t sum_k (y - y*)^2,
     * E = dL/dy = (2/K)(y - y*); the prediction sums y over the window */
    for (int k = 0; k < K; ++k) {
      const double d = y[k] - (k == label ? 1.0 : 0.0);
      E[k] = win ? 2.0 / K * d : 0.0;
      if (win) {
        *loss += d * d / K;
        psum[k] += y[k];
      }
    }
  } else if (net->loss == 0) {
    for (int k = 0; k < K; ++k) {
      const double d = y[k] - target_row[k];
      E[k] = win ? d : 0.0;
      if (win) *loss += 0.5 * d * d;
    }
  } else {
    double mx = y[0];
    for (int k = 1; k < K; ++k) mx = fmax(mx, y[k]);
    double se = 0.0;
    for (int k = 0; k < K; ++k) se += exp(y[k] - mx);
    for (int k = 0; k < K; ++k) {
      const double pi = exp(y[k] - mx) / se;
      E[k] = win ? pi - (k == label ? 1.0 : 0.0) : 0.0;
      if (win) psum[k] += pi;
    }
    if (win) *loss += -(y[label] - mx - log(se));
  }
}

static int check_net(const orc_net *net, const orc_trial *tr) {
  if (!net || !tr || net->n_rec < 1 || net->n_out < 1 || net->n_in < 0 || tr->n_steps < 1) return -1;
  if (net->in.n_src != net->n_in || net->rec.n_src != net->n_rec) return -1;
  if (net->loss == 0 && !tr->target) return -1;
  if ((net->loss == 1 || net->loss == 2) && (tr->label < 0 || tr->label >= net->n_out)) return -1;
  if (net->loss < 0 || net->loss > 2 || net->reset_mode < 0 || net->reset_mode > 1) return -1;
  if (net->etrace_filter < 0 || net->etrace_filter > 2 || (net->etrace_filter == 1 && !(net->tau_e > 0))) return -1;
  if (net->reg_mode < 0 || net->reg_mode > 1 || (net->reg_mode == 1 && !(net->reg_tau > 0))) return -1;
  return 0;
}

int orc_run_trial(const orc_net *net, const orc_trial *tr, int grad_mode, double *g_in,
                  double *g_rec, double *g_out, orc_trace *trace, double *loss_out, int *pred) {
  if (check_net(net, tr)) return -1;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  spikes_t sp;
  if (spikes_init(net, tr, &sp)) { prep_free(&p); return -1; }
  const int T = tr->n_steps, I = net->n_in, J = net->n_rec, K = net->n_out;
  const long nin = net->in.nnz, nrec = net->rec.nnz;
  int rc = -1;

  double *v = calloc(J, sizeof(double)), *a = calloc(J, sizeof(double));
  int *refr = calloc(J, sizeof(int));
  double *y = calloc(K, sizeof(double)), *E = calloc(K, sizeof(double));
  double *psum = calloc(K, sizeof(double));
  /* archived histories, row t (row 0 = zero): psi and L per neuron, E per readout */
  double *psi_h = calloc((size_t)(T + 1) * J, sizeof(double));
  double *L_h = calloc((size_t)(T + 1) * J, sizeof(double));
  double *E_h = calloc((size_t)(T + 1) * K, sizeof(double));
  /* per-synapse traces (eps_v, eps_a, ebar) and, event-driven, the pending arrival */
  long ns = nin + nrec;
  double *ev = calloc(ns + 1, sizeof(double)), *ea = calloc(ns + 1, sizeof(double));
  double *eb = calloc(ns + 1, sizeof(double));
  int *apr = calloc(ns + 1, sizeof(int));
  double *zb = calloc(J, sizeof(double));
  int *apr_o = calloc(J, sizeof(int));
  int *q_src = calloc(ns + 1, sizeof(int));   /* source of each synapse */
  /* time-driven FIFOs of depth d + 1 (eligibility, filtered eligibility, zbar) */
  const int dq1 = net->d_out + 1;
  double *fifo_e = calloc((size_t)(ns + 1) * dq1, sizeof(double)), *fifo_eb = calloc((size_t)(ns + 1) * dq1, sizeof(double));
  double *fifo_z = calloc((size_t)J * dq1, sizeof(double));
  double *esum = calloc(ns + 1, sizeof(double)), *creg = calloc(J, sizeof(double));
  /* moving-average rates f_j^t (eq. ema-rate, row t) and, time-driven, each
   * synapse's G_beta-filtered eligibility (eq. ema-gradient) */
  double *f_h = calloc((size_t)(T + 1) * J, sizeof(double)), *gh = calloc(ns + 1, sizeof(double));
  if (!v || !a || !refr || !y || !E || !psum || !psi_h || !L_h || !E_h || !ev || !ea || !eb ||
      !apr || !zb || !apr_o || !q_src || !fifo_e || !fifo_eb || !fifo_z || !esum || !creg || !f_h || !gh)
    goto done;
  const int ema = net->reg_mode == 1 && net->c_reg != 0.0;
  for (int i = 0; i < net->in.n_src; ++i)
    for (unsigned long r = net->in.row_ptr[i]; r < net->in.row_ptr[i + 1]; ++r) q_src[r] = i;
  for (int i = 0; i < net->rec.n_src; ++i)
    for (unsigned long r = net->rec.row_ptr[i]; r < net->rec.row_ptr[i + 1]; ++r) q_src[nin + (long)r] = i;

  double loss = 0.0;
  /* per-synapse view: target, source kind, source, delay, weight-gradient slot */
#define SYN_TGT(q) ((q) < nin ? (int)net->in.col[q] : (int)net->rec.col[(q)-nin])
#define SYN_G(q) ((q) < nin ? &g_in[q] : &g_rec[(q)-nin])

  for (int t = 1; t <= T; ++t) {
    /* neurons (time-driven) */
    for (int j = 0; j < J; ++j) {
      const double I_t = input_current(net, &p, &sp, j, t);
      const double zprev = sp.zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0;
      const int fz = sp.zforced ? sp.zforced[(long)t * J + j] : -1;
      double psi;
      const int z = neuron_step(net, &p, j, I_t, zprev, fz, &v[j], &a[j], &refr[j], &psi);
      sp.zrec[(long)t * J + j] = (unsigned char)z;
      psi_h[(long)t * J + j] = psi;
      f_h[(long)t * J + j] = p.beta_f * f_h[(long)(t - 1) * J + j] + (1.0 - p.beta_f) * z;
      if (trace) {
        if (trace->v) trace->v[(long)(t - 1) * J + j] = v[j];
        if (trace->a) trace->a[(long)(t - 1) * J + j] = a[j];
        if (trace->psi) trace->psi[(long)(t - 1) * J + j] = psi;
        if (trace->z) trace->z[(long)(t - 1) * J + j] = (unsigned char)z;
      }
    }
    /* readout, error signal, loss */
    readout_step(net, &p, &sp, tr, t, y, E, &loss, psum);
    for (int k = 0; k < K; ++k) E_h[(long)t * K + k] = E[k];
    /* learning signal L_j^t = sum_k B_jk E_k^t (eq. final-gradient) */
    for (int j = 0; j < J; ++j) {
      double Ls = 0.0;
      for (int k = 0; k < K; ++k) Ls = Ls + net->fb[(long)j * K + k] * E[k];
      L_h[(long)t * J + j] = Ls;
    }
    if (trace) {
      for (int k = 0; k < K; ++k) {
        if (trace->y) trace->y[(long)(t - 1) * K + k] = y[k];
        if (trace->err) trace->err[(long)(t - 1) * K + k] = E[k];
      }
      if (trace->learn)
        for (int j = 0; j < J; ++j) trace->learn[(long)(t - 1) * J + j] = L_h[(long)t * J + j];
    }

    if (grad_mode == 1) {
      /* Time-driven gradient computation (Alg. "time-driven gradient
       * computation"): every synapse, every step.  The eligibility of step t
       * enters a FIFO of depth d; the one of step t - d leaves it and meets
       * the learning signal L^t (eq. eprop-approx-final-expanded-subs-
       * rewritten); with a learning-signal delay d^ls, L^t takes part only
       * for t <= T - d^ls (eq. eprop-learning-signal-delay).  The static
       * regularisation term needs the sample's rate and is added at its end
       * from the sum of the dequeued eligibilities. */
      const int dq = net->d_out;
      const double Lon = t <= T - net->d_ls ? 1.0 : 0.0;
      for (long q = 0; q < ns; ++q) {
        const int j = SYN_TGT(q);
        const int kind = q < nin ? 0 : 1;
        const int D = q < nin ? net->in.delay[q] : net->rec.delay[q - nin];
        const double x = spiked(&sp, kind, q_src[q], t - D) ? 1.0 : 0.0;
        const double e = syn_trace(net, &p, x, sp.zrec[(long)(t - 1) * J + j], psi_h[(long)(t - 1) * J + j],
                                   psi_h[(long)t * J + j], neuron_beta(net, j), &ev[q], &ea[q], &eb[q]);
        if (ema) {
          /* Alg. "time-driven gradient computation", moving-average form:
           * c (f_j^s - f*) G_beta(e^s) at s = t - d, for s <= T - d */
          gh[q] = p.beta_f * gh[q] + (1.0 - p.beta_f) * e;
          if (t <= T - dq) *SYN_G(q) += net->c_reg * (f_h[(long)t * J + j] - net->f_target) * gh[q];
        }
        fifo_e[q * (dq + 1) + t % (dq + 1)] = e;
        fifo_eb[q * (dq + 1) + t % (dq + 1)] = eb[q];
        if (t - dq >= 1) {
          *SYN_G(q) += Lon * L_h[(long)t * J + j] * fifo_eb[q * (dq + 1) + (t - dq) % (dq + 1)];
          esum[q] += fifo_e[q * (dq + 1) + (t - dq) % (dq + 1)];
        }
      }
      /* output synapses: zbar = F_kappa(z_j), g_out += E_k^t zbar^{t-d}
       * (eq. eprop-output-new-subs-rewritten) */
      for (int j = 0; j < J; ++j) {
        zb[j] = p.kappa * zb[j] + (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);
        fifo_z[(long)j * (dq + 1) + t % (dq + 1)] = zb[j];
        if (t - dq >= 1)
          for (int k = 0; k < K; ++k)
            g_out[(long)k * J + j] += E[k] * fifo_z[(long)j * (dq + 1) + (t - dq) % (dq + 1)];
      }
    }
  }

  /* static firing-rate regularisation (Methods, "Firing rate regularization"):
   * f_j = (1/T) sum_t z_j^t; loss c/2 sum_j (f_j - f*)^2; per synapse the
   * gradient adds (c/T)(f_j - f*) times the eligibilities paired in the sum */
  for (int j = 0; j < J && net->reg_mode == 0; ++j) {
    double nz = 0.0;
    for (int t = 1; t <= T; ++t) nz += sp.zrec[(long)t * J + j] ? 1.0 : 0.0;
    const double f = nz / T;
    creg[j] = net->c_reg / T * (f - net->f_target);
    loss += 0.5 * net->c_reg * (f - net->f_target) * (f - net->f_target);
  }
  /* moving-average form (eq. sma-loss with the rate of eq. ema-rate):
   * c/2 sum_j sum_t (f_j^t - f*)^2, each neuron's sum formed first (summing
   * 10^5 small terms one by one into the total would lose about 1e-11) */
  for (int j = 0; j < J && net->reg_mode == 1; ++j) {
    double sj = 0.0;
    for (int t = 1; t <= T; ++t) {
      const double df = f_h[(long)t * J + j] - net->f_target;
      sj += df * df;
    }
    loss += 0.5 * net->c_reg * sj;
  }

  if (grad_mode == 1) {
    for (long q = 0; q < ns; ++q) *SYN_G(q) += creg[SYN_TGT(q)] * esum[q];
  } else if (grad_mode == 2) {
    /* Event-driven update (Algs. "event-driven weight update" and its
     * optimized spike-time form), evaluated once the sample is complete, as
     * the event-driven scheme does (Results, "From time-driven to
     * event-driven e-prop"): every synapse with at least one arrival walks
     * the archived history from its first arrival, segment by segment
     * between arrivals, the arrival counted at its segment's first step;
     * eligibility e^s pairs with L^{s+d} (s + d <= T - d^ls) and, for the
     * regularisation, with itself (s <= T - d). */
    const int dq = net->d_out;
    for (int kind = 0; kind < 2; ++kind) {
      const orc_proj *pr = kind == 0 ? &net->in : &net->rec;
      const long base = kind == 0 ? 0 : nin;
      for (int i = 0; i < pr->n_src; ++i)
        for (unsigned long r = pr->row_ptr[i]; r < pr->row_ptr[i + 1]; ++r) {
          const long q = base + (long)r;
          const int j = (int)pr->col[r];
          const int D = pr->delay[r];
          double evq = 0.0, eaq = 0.0, ebq = 0.0, es = 0.0, ghq = 0.0;
          int seg = -1;  /* start of the open segment */
          for (int a = 1; a <= T + 1; ++a) {
            const int arrival = a <= T && spiked(&sp, kind, i, a - D);
            if (!arrival && a <= T) continue;
            if (seg > 0) {
              for (int u = seg; u <= a - 1; ++u) {
                const double e = syn_trace(net, &p, u == seg ? 1.0 : 0.0, sp.zrec[(long)(u - 1) * J + j],
                                           psi_h[(long)(u - 1) * J + j], psi_h[(long)u * J + j], neuron_beta(net, j),
                                           &evq, &eaq, &ebq);
                if (u + dq <= T - net->d_ls) *SYN_G(q) += L_h[(long)(u + dq) * J + j] * ebq;
                if (u <= T - dq) es += e;
                if (ema) {
                  ghq = p.beta_f * ghq + (1.0 - p.beta_f) * e;
                  if (u <= T - dq) *SYN_G(q) += net->c_reg * (f_h[(long)u * J + j] - net->f_target) * ghq;
                }
              }
            }
            seg = a;
          }
          *SYN_G(q) += creg[j] * es;
        }
    }
    for (int j = 0; j < J; ++j) {
      double zbj = 0.0;
      int seg = -1;
      for (int u0 = 1; u0 <= T + 1; ++u0) {
        const int spk = u0 <= T && sp.zrec[(long)u0 * J + j];
        if (!spk && u0 <= T) continue;
        if (seg > 0)
          for (int u = seg; u <= u0 - 1; ++u) {
            zbj = p.kappa * zbj + (u == seg ? 1.0 : 0.0);
            if (u + dq <= T)
              for (int k = 0; k < K; ++k) g_out[(long)k * J + j] += E_h[(long)(u + dq) * K + k] * zbj;
          }
        seg = u0;
      }
    }
  }
#undef SYN_TGT
#undef SYN_G
  if (loss_out) *loss_out = loss;
  if (pred) {
    int best = 0;
    for (int k = 1; k < K; ++k)
      if (psum[k] > psum[best]) best = k;
    *pred = net->loss != 0 ? best : 0;
  }
  rc = 0;
  (void)I;
done:
  free(v); free(a); free(refr); free(y); free(E); free(psum);
  free(psi_h); free(L_h); free(E_h); free(ev); free(ea); free(eb); free(apr); free(zb); free(apr_o);
  free(q_src); free(fifo_e); free(fifo_eb); free(fifo_z); free(esum); free(creg); free(f_h); free(gh);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Forward-mode checks.  A dual number carries a value and its derivative
 * with respect to one seeded weight. */

typedef struct { double x, d; } dual;

static dual dmul_c(double c, dual a) { dual r = {c * a.x, c * a.d}; return r; }
static dual dadd(dual a, dual b) { dual r = {a.x + b.x, a.d + b.d}; return r; }
static dual dsub(dual a, dual b) { dual r = {a.x - b.x, a.d - b.d}; return r; }
static dual dstop(dual a) { dual r = {a.x, 0.0}; return r; }

/* Seeded weight: kind (0 input, 1 recurrent), its source, target and delay. */
typedef struct { int kind, src, tgt, delay; } seed_t;

/* Runs the network over one trial with dual numbers.  If stop_presyn, the
 * spikes of other neurons enter as constants (e-prop's truncation); else
 * their derivatives propagate through the recurrent weights.  Records
 * dz[t*J + j] (t in 0..T) and, if dloss, accumulates the loss tangent
 * sum_t sum_k E_k^t dy_k^t through the readouts. */
static int dual_run(const orc_net *net, const prep_t *p, const spikes_t *sp_ref, const orc_trial *tr,
                    const double *E_rec, seed_t sd, int stop_presyn, double *dz, double *dloss) {
  const int T = tr->n_steps, J = net->n_rec, K = net->n_out;
  dual *v = calloc(J, sizeof(dual)), *a = calloc(J, sizeof(dual)), *y = calloc(K, sizeof(dual));
  int *refr = calloc(J, sizeof(int));
  if (!v || !a || !y || !refr) { free(v); free(a); free(y); free(refr); return -1; }
  memset(dz, 0, sizeof(double) * (size_t)(T + 1) * J);
  double dl = 0.0;
  for (int t = 1; t <= T; ++t) {
    for (int j = 0; j < J; ++j) {
      /* input current with its tangent */
      dual I = {0.0, 0.0};
      for (long q = p->in_ptr[j]; q < p->in_ptr[j + 1]; ++q) {
        const in_syn *s = &p->syn[q];
        const int src_step = t - s->delay;
        const double w = s->kind == 0 ? net->in.w[s->idx] : net->rec.w[s->idx];
        dual zs = {(double)spiked(sp_ref, s->kind, s->src, src_step), 0.0};
        if (s->kind == 1 && !stop_presyn && src_step >= 1) zs.d = dz[(long)src_step * J + s->src];
        dual term = dmul_c(w, zs);
        if (s->kind == sd.kind && s->src == sd.src && j == sd.tgt) term.d += zs.x; /* d(w z)/dw */
        I = dadd(I, term);
      }
      const double beta = neuron_beta(net, j);
      dual zprev = {sp_ref->zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0, dz[(long)(t - 1) * J + j]};
      a[j] = dadd(dmul_c(p->rho, a[j]), zprev);                 /* a^t = rho a + z^{t-1} */
      dual A = dadd((dual){net->v_th, 0.0}, dmul_c(beta, a[j]));  /* adaptive threshold */
      if (net->reset_mode == 1) {
        /* full reset: v^t = alpha v_reset + I after a spike, else alpha v + I */
        v[j] = zprev.x != 0.0 ? dadd((dual){p->alpha * net->v_reset, 0.0}, I) : dadd(dmul_c(p->alpha, v[j]), I);
      } else {
        /* v^t = alpha v + I - z^{t-1} A, with the reset term's derivative stopped */
        dual reset = dstop((dual){zprev.x * A.x, 0.0});
        v[j] = dsub(dadd(dmul_c(p->alpha, v[j]), I), reset);
      }
      const int refractory = refr[j] > 0;
      if (refractory) refr[j] -= 1;
      const double psi = refractory ? 0.0 : surrogate(net, v[j].x - A.x);
      const int z = sp_ref->zrec[(long)t * J + j];   /* same spikes as the reference pass */
      if (z) refr[j] = p->n_ref;
      /* dz/dv = psi, dz/dA = -psi */
      dz[(long)t * J + j] = psi * (v[j].d - A.d);
    }
    if (dloss) {
      /* readout with delay d: y^t = kappa y^{t-1} + W z^{t-d} (eq. leaky_integrator_with_delay) */
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        if (t - net->d_out >= 1)
          for (int j = 0; j < J; ++j) s += net->w_out[(long)k * J + j] * dz[(long)(t - net->d_out) * J + j];
        y[k].d = p->kappa * y[k].d + s;
        dl += E_rec[(long)(t - 1) * K + k] * y[k].d;
      }
    }
  }
  if (dloss && net->c_reg != 0.0 && net->reg_mode == 1) {
    /* tangent of the moving-average regularisation loss:
     * sum_t c (f_j^t - f*) df_j^t, with f and df filtered by eq. ema-rate */
    for (int j = 0; j < J; ++j) {
      double f = 0.0, df = 0.0;
      for (int t = 1; t <= T; ++t) {
        f = p->beta_f * f + (1.0 - p->beta_f) * (sp_ref->zrec[(long)t * J + j] ? 1.0 : 0.0);
        df = p->beta_f * df + (1.0 - p->beta_f) * dz[(long)t * J + j];
        dl += net->c_reg * (f - net->f_target) * df;
      }
    }
  } else if (dloss && net->c_reg != 0.0) {
    /* tangent of the regularisation loss: c (f_j - f*) (1/T) sum_t dz_j^t */
    for (int j = 0; j < J; ++j) {
      double nz = 0.0, sd = 0.0;
      for (int t = 1; t <= T; ++t) {
        nz += sp_ref->zrec[(long)t * J + j] ? 1.0 : 0.0;
        sd += dz[(long)t * J + j];
      }
      dl += net->c_reg * (nz / T - net->f_target) * sd / T;
    }
  }
  if (dloss) *dloss = dl;
  free(v); free(a); free(y); free(refr);
  return 0;
}

/* Runs the reference pass and returns its spikes and error signals. */
static int reference_pass(const orc_net *net, const orc_trial *tr, spikes_t *sp, double **E_rec) {
  const int T = tr->n_steps, J = net->n_rec, K = net->n_out;
  unsigned char *z = calloc((size_t)T * J, 1);
  *E_rec = calloc((size_t)T * K, sizeof(double));
  orc_trace trc;
  memset(&trc, 0, sizeof(trc));
  trc.z = z;
  trc.err = *E_rec;
  double loss;
  if (!z || !*E_rec || orc_run_trial(net, tr, 0, NULL, NULL, NULL, &trc, &loss, NULL) ||
      spikes_init(net, tr, sp)) {
    free(z); free(*E_rec); *E_rec = NULL;
    return -1;
  }
  for (int t = 1; t <= T; ++t)
    for (int j = 0; j < J; ++j) sp->zrec[(long)t * J + j] = z[(long)(t - 1) * J + j];
  free(z);
  return 0;
}

static void for_each_weight(const orc_net *net, int kind, long q, seed_t *sd) {
  const orc_proj *pr = kind == 0 ? &net->in : &net->rec;
  int src = 0;
  while (pr->row_ptr[src + 1] <= (unsigned long)q) ++src;
  sd->kind = kind;
  sd->src = src;
  sd->tgt = (int)pr->col[q];
  sd->delay = pr->delay[q];
}

int orc_bruteforce_eprop(const orc_net *net, const orc_trial *tr, double *g_in, double *g_rec) {
  if (check_net(net, tr)) return -1;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  spikes_t sp;
  double *E_rec = NULL;
  if (reference_pass(net, tr, &sp, &E_rec)) { prep_free(&p); return -1; }
  const int T = tr->n_steps, J = net->n_rec, K = net->n_out;
  double *dz = calloc((size_t)(T + 1) * J, sizeof(double));
  int rc = dz ? 0 : -1;
  for (int kind = 0; kind < 2 && rc == 0; ++kind) {
    const orc_proj *pr = kind == 0 ? &net->in : &net->rec;
    for (long q = 0; q < pr->nnz && rc == 0; ++q) {
      seed_t sd;
      for_each_weight(net, kind, q, &sd);
      rc = dual_run(net, &p, &sp, tr, E_rec, sd, 1, dz, NULL);
      /* eq. summation-future, with the readout delay d
       * (eq. eprop-approx-final-expanded) and the learning-signal delay d^ls
       * (eq. eprop-learning-signal-delay):
       * sum_{t'<=T-d} [sum_k B_jk sum_{t'+d<=t<=T-d^ls} E_k^t kappa^(t-d-t')] e^t',
       * plus the static regularisation (c/T)(f_j - f*) sum_{t'<=T-d} e^t' */
      const int d = net->d_out;
      double g = 0.0, es = 0.0;
      for (int tp = 1; tp <= T - d; ++tp) {
        double Ls = 0.0;
        for (int k = 0; k < K; ++k) {
          double fut = 0.0;
          for (int t = tp + d; t <= T - net->d_ls; ++t) fut += E_rec[(long)(t - 1) * K + k] * pow(p.kappa_e, t - d - tp);
          Ls += net->fb[(long)sd.tgt * K + k] * fut;
        }
        g += Ls * dz[(long)tp * J + sd.tgt];
        es += dz[(long)tp * J + sd.tgt];
      }
      if (net->reg_mode == 1) {
        /* moving-average regulariser: sum_{s<=T-d} c (f^s - f*) sum_{s'<=s} (1-beta) beta^(s-s') e^s' */
        double f = 0.0;
        for (int s2 = 1; s2 <= T - d; ++s2) {
          f = p.beta_f * f + (1.0 - p.beta_f) * (sp.zrec[(long)s2 * J + sd.tgt] ? 1.0 : 0.0);
          double G = 0.0;
          for (int s1 = 1; s1 <= s2; ++s1) G += (1.0 - p.beta_f) * pow(p.beta_f, s2 - s1) * dz[(long)s1 * J + sd.tgt];
          g += net->c_reg * (f - net->f_target) * G;
        }
      } else {
        double nz = 0.0;
        for (int t = 1; t <= T; ++t) nz += sp.zrec[(long)t * J + sd.tgt] ? 1.0 : 0.0;
        g += net->c_reg / T * (nz / T - net->f_target) * es;
      }
      (kind == 0 ? g_in : g_rec)[q] = g;
    }
  }
  free(dz);
  free(E_rec);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

int orc_forward_mode_loss_grad(const orc_net *net, const orc_trial *tr, double *g_in, double *g_rec) {
  if (check_net(net, tr)) return -1;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  spikes_t sp;
  double *E_rec = NULL;
  if (reference_pass(net, tr, &sp, &E_rec)) { prep_free(&p); return -1; }
  const int T = tr->n_steps, J = net->n_rec;
  double *dz = calloc((size_t)(T + 1) * J, sizeof(double));
  int rc = dz ? 0 : -1;
  for (int kind = 0; kind < 2 && rc == 0; ++kind) {
    const orc_proj *pr = kind == 0 ? &net->in : &net->rec;
    for (long q = 0; q < pr->nnz && rc == 0; ++q) {
      seed_t sd;
      double dl = 0.0;
      for_each_weight(net, kind, q, &sd);
      rc = dual_run(net, &p, &sp, tr, E_rec, sd, 0, dz, &dl);
      (kind == 0 ? g_in : g_rec)[q] = dl;
    }
  }
  free(dz);
  free(E_rec);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

/* ------------------------------------------------------------------------ */

int orc_forced_sampled(const orc_net *net, const orc_trial *tr, int n_sample, const int *targets,
                       double *g_in, double *g_rec, double *psi_out, double *loss_out) {
  if (check_net(net, tr) || !tr->forced) return -1;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  spikes_t sp;
  if (spikes_init(net, tr, &sp)) { prep_free(&p); return -1; }
  const int T = tr->n_steps, J = net->n_rec, K = net->n_out;
  /* forced spikes are the recurrent spike train */
  memcpy(sp.zrec, sp.zforced, (size_t)(T + 1) * J);
  double *y = calloc(K, sizeof(double)), *E = calloc(K, sizeof(double)), *psum = calloc(K, sizeof(double));
  double *E_h = calloc((size_t)(T + 1) * K, sizeof(double));
  double *psi_h = calloc((size_t)(T + 1), sizeof(double)), *L_h = calloc((size_t)(T + 1), sizeof(double));
  int rc = (y && E && psum && E_h && psi_h && L_h) ? 0 : -1;
  double loss = 0.0;
  for (int t = 1; t <= T && rc == 0; ++t) {
    readout_step(net, &p, &sp, tr, t, y, E, &loss, psum);
    for (int k = 0; k < K; ++k) E_h[(long)t * K + k] = E[k];
  }
  for (int j = 0; j < J; ++j) {  /* rate regularisation of every neuron */
    double nz = 0.0, f = 0.0, sf = 0.0;
    for (int t = 1; t <= T; ++t) {
      const double z = sp.zrec[(long)t * J + j] ? 1.0 : 0.0;
      nz += z;
      f = p.beta_f * f + (1.0 - p.beta_f) * z;
      sf += (f - net->f_target) * (f - net->f_target);
    }
    if (net->reg_mode == 1) loss += 0.5 * net->c_reg * sf;
    if (net->reg_mode == 0) loss += 0.5 * net->c_reg * (nz / T - net->f_target) * (nz / T - net->f_target);
  }
  for (int n = 0; n < n_sample && rc == 0; ++n) {
    const int j = targets[n];
    if (j < 0 || j >= J) { rc = -1; break; }
    double v = 0.0, a = 0.0;
    int refr = 0;
    for (int t = 1; t <= T; ++t) {
      const double I_t = input_current(net, &p, &sp, j, t);
      const double zprev = sp.zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0;
      double psi;
      neuron_step(net, &p, j, I_t, zprev, sp.zrec[(long)t * J + j], &v, &a, &refr, &psi);
      psi_h[t] = psi;
      if (psi_out) psi_out[(long)n * T + (t - 1)] = psi;
      double Ls = 0.0;
      for (int k = 0; k < K; ++k) Ls = Ls + net->fb[(long)j * K + k] * E_h[(long)t * K + k];
      L_h[t] = Ls;
    }
    double nz = 0.0;
    for (int t = 1; t <= T; ++t) nz += sp.zrec[(long)t * J + j] ? 1.0 : 0.0;
    const double creg = net->reg_mode == 0 ? net->c_reg / T * (nz / T - net->f_target) : 0.0;
    for (long q = p.in_ptr[j]; q < p.in_ptr[j + 1]; ++q) {
      const in_syn *s = &p.syn[q];
      double ev = 0.0, ea = 0.0, eb = 0.0, g = 0.0, es = 0.0, gh = 0.0, f = 0.0;
      for (int t = 1; t <= T; ++t) {
        const double e = syn_trace(net, &p, spiked(&sp, s->kind, s->src, t - s->delay) ? 1.0 : 0.0,
                                   sp.zrec[(long)(t - 1) * J + j], psi_h[t - 1], psi_h[t], neuron_beta(net, j),
                                   &ev, &ea, &eb);
        if (t + net->d_out <= T - net->d_ls) g += L_h[t + net->d_out] * eb;
        if (t <= T - net->d_out) es += e;
        if (net->reg_mode == 1 && net->c_reg != 0.0) {
          f = p.beta_f * f + (1.0 - p.beta_f) * (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);
          gh = p.beta_f * gh + (1.0 - p.beta_f) * e;
          if (t <= T - net->d_out) g += net->c_reg * (f - net->f_target) * gh;
        }
      }
      (s->kind == 0 ? g_in : g_rec)[s->idx] = g + creg * es;
    }
  }
  if (loss_out) *loss_out = loss;
  free(y); free(E); free(psum); free(E_h); free(psi_h); free(L_h);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Bounds for checking an FP32 evaluation of a teacher-forced trial (see the
 * header), by running error analysis: a computed quantity x carries mu(x)
 * with |fl(x) - x| <= u mu(x) to first order in u = 2^-24; one rounding per
 * operation, so z = x op y gives mu(z) = (mu of the operands, propagated) +
 * |z|, and a constant rounded to FP32 adds its own magnitude. */

static const double kU32 = 5.9604644775390625e-08;   /* 2^-24 */

int orc_fp32_bounds(const orc_net *net, const orc_trial *tr, double quantum, const double *psi_given, int n_sample,
                    const int *targets, double *psi_own, double *psi_bound, double *g_in, double *g_rec,
                    double *g_out, double *b_in, double *b_rec, double *b_out) {
  if (check_net(net, tr) || !tr->forced || !(quantum >= 0.0)) return -1;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  spikes_t sp;
  if (spikes_init(net, tr, &sp)) { prep_free(&p); return -1; }
  const int T = tr->n_steps, J = net->n_rec, K = net->n_out, d = net->d_out;
  const int ema = net->reg_mode == 1 && net->c_reg != 0.0;
  const double u = kU32, cs = 7.0;   /* cs: roundings downstream of psi, in units of u (header) */
  memcpy(sp.zrec, sp.zforced, (size_t)(T + 1) * J);
  double *y = calloc(K, sizeof(double)), *E = calloc(K, sizeof(double)), *psum = calloc(K, sizeof(double));
  double *E_h = calloc((size_t)(T + 1) * K, sizeof(double));
  double *psi_h = calloc((size_t)(T + 1), sizeof(double));
  double *L_h = calloc((size_t)(T + 1), sizeof(double)), *La_h = calloc((size_t)(T + 1), sizeof(double));
  double *f_h = calloc((size_t)(T + 1), sizeof(double));
  int rc = (y && E && psum && E_h && psi_h && L_h && La_h && f_h) ? 0 : -1;
  double loss = 0.0;
  for (int t = 1; t <= T && rc == 0; ++t) {
    readout_step(net, &p, &sp, tr, t, y, E, &loss, psum);
    for (int k = 0; k < K; ++k) E_h[(long)t * K + k] = E[k];
  }
  /* output synapses (eq. eprop-output-new-subs-rewritten): sum over t of
   * E_k^{t+d} zbar_j^t; every term has the sign of E, so the rounding bound
   * is cs u sum_t |E_k^{t+d}| zbar_j^t */
  for (int j = 0; j < J && rc == 0 && (g_out || b_out); ++j) {
    double zb = 0.0, g[64] = {0}, b[64] = {0};
    for (int t = 1; t + d <= T; ++t) {
      zb = p.kappa * zb + (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);
      for (int k = 0; k < K && k < 64; ++k) {
        g[k] += E_h[(long)(t + d) * K + k] * zb;
        b[k] += cs * u * fabs(E_h[(long)(t + d) * K + k]) * zb;
      }
    }
    for (int k = 0; k < K && k < 64; ++k) {
      if (g_out) g_out[(long)k * J + j] = g[k];
      if (b_out) b_out[(long)k * J + j] = b[k];
    }
  }
  const int ns = n_sample < 0 ? J : n_sample;
  for (int n = 0; n < ns && rc == 0; ++n) {
    const int j = n_sample < 0 ? n : targets[n];
    if (j < 0 || j >= J) { rc = -1; break; }
    const double beta = neuron_beta(net, j);
    /* the neuron's recursion in FP64 and the running bound of its FP32 evaluation */
    double v = 0.0, a = 0.0, mu_v = 0.0, mu_a = 0.0;
    int refr = 0;
    for (int t = 1; t <= T; ++t) {
      const double v_prev = v, a_prev = a;
      const int refr_prev = refr;
      const double I_t = input_current(net, &p, &sp, j, t);
      int n_arr = 0;
      for (long q = p.in_ptr[j]; q < p.in_ptr[j + 1]; ++q)
        n_arr += spiked(&sp, p.syn[q].kind, p.syn[q].src, t - p.syn[q].delay);
      const double zprev = sp.zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0;
      double psi;
      neuron_step(net, &p, j, I_t, zprev, sp.zrec[(long)t * J + j], &v, &a, &refr, &psi);
      /* a = rho a + z (rho rounded, product, sum); A = v_th + beta a (v_th, beta rounded) */
      double A = net->v_th, mu_A = fabs(net->v_th);
      if (beta != 0.0) {
        mu_a = p.rho * mu_a + 2.0 * fabs(p.rho * a_prev) + fabs(a);
        A = net->v_th + beta * a;
        mu_A = fabs(net->v_th) + beta * mu_a + 2.0 * fabs(beta * a) + fabs(A);
      }
      /* the input current: the arriving weights summed exactly and rounded
       * once, plus `quantum` per arriving weight */
      const double mu_I = fabs(I_t) + n_arr * quantum / u;
      if (net->reset_mode == 1 && zprev != 0.0)   /* alpha v_reset + I: alpha, v_reset, product, sum */
        mu_v = 3.0 * fabs(p.alpha * net->v_reset) + mu_I + fabs(v);
      else                                         /* (alpha v + I) - z A */
        mu_v = p.alpha * mu_v + 2.0 * fabs(p.alpha * v_prev) + mu_I + fabs(p.alpha * v_prev + I_t) +
               zprev * mu_A + fabs(v);
      double mu_psi = 0.0;
      if (refr_prev == 0) {   /* psi = 0 exactly while refractory */
        const double dv = v - A, mu_dv = mu_v + mu_A + fabs(dv);
        if (net->surrogate == 1)   /* gamma exp(-beta |dv|): the exponent's error, exp, gamma, beta, products */
          mu_psi = psi * (net->sg_beta * mu_dv + 2.0 * net->sg_beta * fabs(dv) + 4.0);
        else                       /* gamma max(0, 1 - beta |dv|): Lipschitz gamma beta, and its own roundings */
          mu_psi = net->sg_gamma * net->sg_beta * mu_dv + 3.0 * net->sg_gamma;
      }
      if (psi_own) psi_own[(long)n * T + (t - 1)] = psi;
      if (psi_bound) psi_bound[(long)n * T + (t - 1)] = u * mu_psi;
      psi_h[t] = psi_given ? psi_given[(long)n * T + (t - 1)] : psi;
      double Ls = 0.0, La = 0.0;
      for (int k = 0; k < K; ++k) {
        Ls = Ls + net->fb[(long)j * K + k] * E_h[(long)t * K + k];
        La = La + fabs(net->fb[(long)j * K + k] * E_h[(long)t * K + k]);
      }
      L_h[t] = Ls;
      La_h[t] = La;
      f_h[t] = p.beta_f * f_h[t - 1] + (1.0 - p.beta_f) * (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);
    }
    double nz = 0.0;
    for (int t = 1; t <= T; ++t) nz += sp.zrec[(long)t * J + j] ? 1.0 : 0.0;
    const double creg = net->reg_mode == 0 ? net->c_reg / T * (nz / T - net->f_target) : 0.0;
    /* Alg. "time-driven gradient computation" on the archived psi history, as
     * orc_forced_sampled, with the same recursion run on absolute values for
     * the rounding bound */
    for (long q = p.in_ptr[j]; q < p.in_ptr[j + 1]; ++q) {
      const in_syn *s = &p.syn[q];
      double ev = 0.0, ea = 0.0, eb = 0.0, gh = 0.0, g = 0.0, es = 0.0;
      double ea_abs = 0.0, eb_abs = 0.0, gh_abs = 0.0, s_eabs = 0.0, bnd = 0.0;
      for (int t = 1; t <= T; ++t) {
        const double ev_prev = ev;
        const double zp = sp.zrec[(long)(t - 1) * J + j];
        const double e = syn_trace(net, &p, spiked(&sp, s->kind, s->src, t - s->delay) ? 1.0 : 0.0, zp, psi_h[t - 1],
                                   psi_h[t], beta, &ev, &ea, &eb);
        ea_abs = psi_h[t - 1] * fabs(ev_prev) + fabs(p.rho - psi_h[t - 1] * beta) * ea_abs;
        const double e_abs = psi_h[t] * (fabs(ev) + beta * ea_abs);
        eb_abs = p.kappa_e * eb_abs + e_abs;
        if (t + d <= T - net->d_ls) {
          g += L_h[t + d] * eb;
          bnd += cs * u * La_h[t + d] * eb_abs;
        }
        if (t <= T - d) {
          es += e;
          s_eabs += e_abs;
        }
        if (ema) {
          gh = p.beta_f * gh + (1.0 - p.beta_f) * e;
          gh_abs = p.beta_f * gh_abs + (1.0 - p.beta_f) * e_abs;
          if (t <= T - d) {
            const double df = f_h[t] - net->f_target;
            g += net->c_reg * df * gh;
            bnd += net->c_reg * (cs * u * fabs(df) + u * fabs(f_h[t])) * gh_abs;
          }
        }
      }
      if (g_in && g_rec) (s->kind == 0 ? g_in : g_rec)[s->idx] = g + creg * es;
      if (b_in && b_rec) (s->kind == 0 ? b_in : b_rec)[s->idx] = bnd + cs * u * fabs(creg) * s_eabs;
    }
  }
  free(y); free(E); free(psum); free(E_h); free(psi_h); free(L_h); free(La_h); free(f_h);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* e-prop+ update schedule: weight updates at every spike over a continuous
 * run (see the header). */

typedef struct {
  double ev, ea, eb, gh;   /* eligibility vector, filtered trace, G_beta-filtered trace */
  double ea_a, eb_a, gh_a; /* the same recursions on the absolute values of their terms */
  int s_done;              /* last eligibility step already used */
  int last;                /* last arrival at or before s_done (0: none) */
} online_syn;

/* Advances one synapse (source kind/src, delay D, target j) over the
 * eligibility steps s_done+1 .. s_new and returns the gradient they carry:
 * sum_s L_j^{s+d} ebar^s + c (f_j^s - f*) G_beta(e^s) (Alg. "event-driven
 * weight update", steps of the left-open interval). */
static double online_walk(const orc_net *net, const prep_t *p, const spikes_t *sp, int kind, int src, int D, int j,
                          online_syn *st, int s_new, int cutoff, const double *psi_h, const double *L_h,
                          const double *La_h, const double *f_h, double *gabs) {
  const int J = net->n_rec;
  const int ema = net->reg_mode == 1 && net->c_reg != 0.0;
  const double beta = neuron_beta(net, j);
  double g = 0.0;
  for (int s = st->s_done + 1; s <= s_new; ++s) {
    const int x = spiked(sp, kind, src, s - D);
    if (x) st->last = s;
    if (cutoff > 0 && (st->last == 0 || s - st->last >= cutoff)) {
      /* beyond the cutoff the traces count as decayed */
      st->ev = st->ea = st->eb = st->gh = 0.0;
      st->ea_a = st->eb_a = st->gh_a = 0.0;
      continue;
    }
    const double ev_prev = st->ev, pp = psi_h[(long)(s - 1) * J + j], pn = psi_h[(long)s * J + j];
    const double e = syn_trace(net, p, x ? 1.0 : 0.0, sp->zrec[(long)(s - 1) * J + j], pp, pn, beta, &st->ev,
                               &st->ea, &st->eb);
    st->gh = p->beta_f * st->gh + (1.0 - p->beta_f) * e;
    g += L_h[(long)(s + net->d_out) * J + j] * st->eb;
    if (ema) g += net->c_reg * (f_h[(long)s * J + j] - net->f_target) * st->gh;
    /* the absolute term sum of the same gradient (for bounding an FP32 evaluation) */
    st->ea_a = pp * fabs(ev_prev) + fabs(p->rho - pp * beta) * st->ea_a;
    const double e_a = pn * (fabs(st->ev) + beta * st->ea_a);
    st->eb_a = p->kappa_e * st->eb_a + e_a;
    st->gh_a = p->beta_f * st->gh_a + (1.0 - p->beta_f) * e_a;
    *gabs += La_h[(long)(s + net->d_out) * J + j] * st->eb_a;
    if (ema) *gabs += net->c_reg * (fabs(f_h[(long)s * J + j] - net->f_target) + fabs(f_h[(long)s * J + j])) * st->gh_a;
  }
  if (s_new > st->s_done) st->s_done = s_new;
  return g;
}

/* The readout side: zbar_j^r = kappa zbar_j^{r-1} + z_j^r over r_done+1 ..
 * r_new, each r adding E_k^{r+d} zbar_j^r to g[k]
 * (eq. eprop-output-new-subs-rewritten), with the same cutoff rule. */
static void online_walk_out(const orc_net *net, const prep_t *p, const spikes_t *sp, int j, double *zb, int *r_done,
                            int *last, int r_new, int cutoff, const double *E_h, double *g, double *gabs) {
  const int J = net->n_rec, K = net->n_out;
  for (int r = *r_done + 1; r <= r_new; ++r) {
    const int x = sp->zrec[(long)r * J + j];
    if (x) *last = r;
    if (cutoff > 0 && (*last == 0 || r - *last >= cutoff)) {
      *zb = 0.0;
      continue;
    }
    *zb = p->kappa * *zb + (x ? 1.0 : 0.0);
    for (int k = 0; k < K; ++k) {
      g[k] += E_h[(long)(r + net->d_out) * K + k] * *zb;
      gabs[k] += fabs(E_h[(long)(r + net->d_out) * K + k]) * *zb;
    }
  }
  if (r_new > *r_done) *r_done = r_new;
}

int orc_run_online(const orc_net *net0, int n_samples, const orc_trial *smp, double eta, int cutoff,
                   int flush, double *w_in, double *w_rec, double *w_out, double *g_in, double *g_rec,
                   double *g_out, double *loss_out, unsigned char *z_out, double *a_in, double *a_rec,
                   double *a_out) {
  if (!net0 || !smp || n_samples < 1 || !w_in || !w_rec || !w_out || !loss_out || cutoff < 0) return -1;
  if (net0->c_reg != 0.0 && net0->reg_mode != 1) return -1;
  orc_net nt = *net0;  /* the same network, reading the weights being trained */
  nt.in.w = w_in;
  nt.rec.w = w_rec;
  nt.w_out = w_out;
  const orc_net *net = &nt;
  long Tt = 0;
  for (int k = 0; k < n_samples; ++k) {
    if (check_net(net, &smp[k]) || smp[k].forced != smp[0].forced) return -1;
    Tt += smp[k].n_steps;
  }
  if (Tt > 1000000) return -1;
  const int T = (int)Tt, I = net->n_in, J = net->n_rec, K = net->n_out;
  prep_t p;
  if (prep_init(net, &p)) return -1;
  /* the run's spike record: sample k's steps are off_k + 1 .. off_k + T_k */
  spikes_t sp;
  memset(&sp, 0, sizeof(sp));
  sp.T = T;
  sp.I = I;
  sp.J = J;
  int *off = calloc((size_t)n_samples + 1, sizeof(int)), *smp_of = calloc((size_t)T + 1, sizeof(int));
  sp.zin = calloc((size_t)T * (I > 0 ? I : 1), 1);
  sp.list = calloc((size_t)J, sizeof(int));
  sp.zrec = calloc((size_t)(T + 1) * J, 1);
  if (smp[0].forced) sp.zforced = calloc((size_t)(T + 1) * J, 1);
  double *v = calloc(J, sizeof(double)), *a = calloc(J, sizeof(double)), *y = calloc(K, sizeof(double));
  double *E = calloc(K, sizeof(double)), *psum = calloc(K, sizeof(double)), *gk = calloc(K, sizeof(double));
  double *gka = calloc(K, sizeof(double));
  int *refr = calloc(J, sizeof(int));
  double *psi_h = calloc((size_t)(T + 1) * J, sizeof(double)), *L_h = calloc((size_t)(T + 1) * J, sizeof(double));
  double *La_h = calloc((size_t)(T + 1) * J, sizeof(double));   /* sum_k |B_jk E_k^t| */
  double *f_h = calloc((size_t)(T + 1) * J, sizeof(double)), *E_h = calloc((size_t)(T + 1) * K, sizeof(double));
  const long nin = net->in.nnz, ns = net->in.nnz + net->rec.nnz;
  online_syn *syn = calloc((size_t)ns + 1, sizeof(online_syn));
  double *zbo = calloc(J, sizeof(double));
  int *r_done = calloc(J, sizeof(int)), *zlast = calloc(J, sizeof(int));
  int rc = -1;
  if (!off || !smp_of || !sp.zin || !sp.list || !sp.zrec || (smp[0].forced && !sp.zforced) || !v || !a || !y || !E || !psum ||
      !gk || !gka || !refr || !psi_h || !L_h || !La_h || !f_h || !E_h || !syn || !zbo || !r_done || !zlast)
    goto done;
  for (int k = 0; k < n_samples; ++k) {
    off[k + 1] = off[k] + smp[k].n_steps;
    for (int t = off[k] + 1; t <= off[k + 1]; ++t) smp_of[t] = k;
    for (long e = 0; e < smp[k].n_in_spikes; ++e) {
      const unsigned int s0 = smp[k].in_step[e], i = smp[k].in_src[e];
      if ((int)s0 >= smp[k].n_steps || (int)i >= I) goto done;
      sp.zin[(long)(off[k] + s0) * I + i] = 1;
    }
    for (long e = 0; smp[k].forced && e < smp[k].n_forced; ++e) {
      const unsigned int t0 = smp[k].forced_step[e], j = smp[k].forced_neuron[e];
      if (t0 < 1 || (int)t0 > smp[k].n_steps || (int)j >= J) goto done;
      sp.zforced[(long)(off[k] + t0) * J + j] = 1;
    }
  }
  for (int k = 0; k < n_samples; ++k) loss_out[k] = 0.0;
  const int d = net->d_out, lag = 1 + net->d_ls + net->d_out;
  for (int t = 1; t <= T; ++t) {
    const int k = smp_of[t], lt = t - off[k];
    const orc_trial *tr = &smp[k];
    for (int j = 0; j < J; ++j) {
      /* arrivals at t: update first, then deliver with the new weight
       * (eq. lif_update's input sums, canonical order) */
      double I_t = 0.0;
      for (long q = p.in_ptr[j]; q < p.in_ptr[j + 1]; ++q) {
        const in_syn *si = &p.syn[q];
        if (!spiked(&sp, si->kind, si->src, t - si->delay)) continue;
        const long sq = si->kind == 0 ? si->idx : nin + si->idx;
        double ga = 0.0;
        const double g = online_walk(net, &p, &sp, si->kind, si->src, si->delay, j, &syn[sq], t - lag, cutoff, psi_h,
                                     L_h, La_h, f_h, &ga);
        double *w = si->kind == 0 ? &w_in[si->idx] : &w_rec[si->idx];
        *w = *w - eta * g;
        if (si->kind == 0 && a_in) a_in[si->idx] += fabs(eta) * ga;
        if (si->kind == 1 && a_rec) a_rec[si->idx] += fabs(eta) * ga;
        if (si->kind == 0 && g_in) g_in[si->idx] += g;
        if (si->kind == 1 && g_rec) g_rec[si->idx] += g;
        I_t = I_t + *w;
      }
      const double zprev = sp.zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0;
      const int fz = sp.zforced ? sp.zforced[(long)t * J + j] : -1;
      double psi;
      const int z = neuron_step(net, &p, j, I_t, zprev, fz, &v[j], &a[j], &refr[j], &psi);
      sp.zrec[(long)t * J + j] = (unsigned char)z;
      psi_h[(long)t * J + j] = psi;
      f_h[(long)t * J + j] = p.beta_f * f_h[(long)(t - 1) * J + j] + (1.0 - p.beta_f) * z;
      if (z_out) z_out[(long)(t - 1) * J + j] = (unsigned char)z;
    }
    /* readout synapses whose presynaptic spike arrives now */
    for (int j = 0; j < J && t - d >= 1; ++j) {
      if (!sp.zrec[(long)(t - d) * J + j]) continue;
      for (int kk = 0; kk < K; ++kk) gk[kk] = gka[kk] = 0.0;
      online_walk_out(net, &p, &sp, j, &zbo[j], &r_done[j], &zlast[j], t - 1 - d, cutoff, E_h, gk, gka);
      for (int kk = 0; kk < K; ++kk) {
        w_out[(long)kk * J + j] -= eta * gk[kk];
        if (g_out) g_out[(long)kk * J + j] += gk[kk];
        if (a_out) a_out[(long)kk * J + j] += fabs(eta) * gka[kk];
      }
    }
    readout_core(net, &p, &sp, t, tr->target ? tr->target + (long)(lt - 1) * K : NULL,
                 tr->window ? tr->window[lt - 1] : 1, tr->label, y, E, &loss_out[k], psum);
    for (int kk = 0; kk < K; ++kk) E_h[(long)t * K + kk] = E[kk];
    double sreg = 0.0;  /* this step's moving-average regulariser, summed before the total */
    for (int j = 0; j < J; ++j) {
      double Ls = 0.0, La = 0.0;
      for (int kk = 0; kk < K; ++kk) {
        Ls = Ls + net->fb[(long)j * K + kk] * E[kk];
        La = La + fabs(net->fb[(long)j * K + kk] * E[kk]);
      }
      L_h[(long)t * J + j] = Ls;
      La_h[(long)t * J + j] = La;
      const double df = f_h[(long)t * J + j] - net->f_target;
      sreg += df * df;
    }
    if (net->reg_mode == 1 && net->c_reg != 0.0) loss_out[k] += 0.5 * net->c_reg * sreg;
  }
  if (flush) {
    /* as if a spike arrived at every synapse after the last step */
    for (int kind = 0; kind < 2; ++kind) {
      const orc_proj *pr = kind == 0 ? &net->in : &net->rec;
      for (int i = 0; i < pr->n_src; ++i)
        for (unsigned long r = pr->row_ptr[i]; r < pr->row_ptr[i + 1]; ++r) {
          const long sq = kind == 0 ? (long)r : nin + (long)r;
          double ga = 0.0;
          const double g = online_walk(net, &p, &sp, kind, i, pr->delay[r], (int)pr->col[r], &syn[sq], T + 1 - lag,
                                       cutoff, psi_h, L_h, La_h, f_h, &ga);
          (kind == 0 ? w_in : w_rec)[r] -= eta * g;
          if (a_in && kind == 0) a_in[r] += fabs(eta) * ga;
          if (a_rec && kind == 1) a_rec[r] += fabs(eta) * ga;
          if (kind == 0 && g_in) g_in[r] += g;
          if (kind == 1 && g_rec) g_rec[r] += g;
        }
    }
    for (int j = 0; j < J; ++j) {
      for (int kk = 0; kk < K; ++kk) gk[kk] = gka[kk] = 0.0;
      online_walk_out(net, &p, &sp, j, &zbo[j], &r_done[j], &zlast[j], T - d, cutoff, E_h, gk, gka);
      for (int kk = 0; kk < K; ++kk) {
        w_out[(long)kk * J + j] -= eta * gk[kk];
        if (g_out) g_out[(long)kk * J + j] += gk[kk];
        if (a_out) a_out[(long)kk * J + j] += fabs(eta) * gka[kk];
      }
    }
  }
  rc = 0;
done:
  free(off); free(smp_of); free(v); free(a); free(y); free(E); free(psum); free(gk); free(gka); free(refr);
  free(psi_h); free(L_h); free(La_h); free(f_h); free(E_h); free(syn); free(zbo); free(r_done); free(zlast);
  spikes_free(&sp);
  prep_free(&p);
  return rc;
}

/* Gradient descent (eq. gradient-descent) on the mini-batch mean, or Adam
 * with eq. eta-adam-fast and eq. delta-w-adam-fast applied once per
 * iteration to the mini-batch mean gradient. */
void orc_apply(long n, double *w, const double *g_sum, double n_trials, int optimizer, double eta,
               double beta1, double beta2, double eps_hat, long step, double *m, double *v) {
  const double eta_t = eta * sqrt(1.0 - pow(beta2, (double)step)) / (1.0 - pow(beta1, (double)step));
  for (long i = 0; i < n; ++i) {
    const double G = g_sum[i] / n_trials;
    if (optimizer == 0) {
      w[i] = w[i] - eta * G;
    } else {
      m[i] = beta1 * m[i] + (1.0 - beta1) * G;
      v[i] = beta2 * v[i] + (1.0 - beta2) * G * G;
      w[i] = w[i] - eta_t * m[i] / (sqrt(v[i]) + eps_hat);
    }
  }
}
