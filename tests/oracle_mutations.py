"""Planted-mistake check of the oracle's pins (CPU only, a few minutes).

Each entry below plants one plausible mistake in a copy of the oracle's C
source: a dropped term, a wrong sign, a swapped operand or index, an
off-by-one delay, a wrong filter constant, an optimiser slip.  The pins in
tests/test_oracle.py must fail for every one of them; a mistake that
survives marks a part of the oracle that no pin holds.

Run: python tests/oracle_mutations.py [-j WORKERS] [NAME ...]
Exit status 0 when every planted mistake is caught (the pins are first run
on an unchanged copy, which must pass).

Not collected by pytest (its name has no test_ prefix): each entry rebuilds
the oracle and runs the whole pin suite.
"""
import argparse
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join("oracle", "eprop_oracle.c")

# (name, passage the correct line follows, correct text, planted mistake)
MUTATIONS = [
    # neuron dynamics (Methods, "Neuron models")
    ("adaptation_leak", "eq. spike-threshold-adaptation",
     "*a = p->rho * *a + zprev;", "*a = p->rho * *a + (1.0 - p->rho) * zprev;"),
    ("threshold_from_spike", "adaptive threshold",
     "const double A = net->v_th + beta * *a;", "const double A = net->v_th + beta * zprev;"),
    ("reset_by_v_th", "eq. lif_update",
     "else *v = p->alpha * *v + I - zprev * A;", "else *v = p->alpha * *v + I - zprev * net->v_th;"),
    ("tie_does_not_spike", "eq. binary-spike-state-variable",
     "z = (!refractory && *v >= A) ? 1 : 0;", "z = (!refractory && *v > A) ? 1 : 0;"),
    ("psi_while_refractory", "surrogate, zero while refractory",
     "*psi = refractory ? 0.0 : surrogate(net, *v - A);", "*psi = surrogate(net, *v - A);"),
    ("refractory_one_long", "refractory period",
     "if (z) *refr = p->n_ref;\n  return z;", "if (z) *refr = p->n_ref + 1;\n  return z;"),
    ("full_reset_leaks", "full reset (Results, \"Continuous dynamics\")",
     "if (net->reset_mode == 1) *v = p->alpha * (zprev != 0.0 ? net->v_reset : *v) + I;",
     "if (net->reset_mode == 1) *v = (zprev != 0.0 ? net->v_reset : p->alpha * *v) + I;"),
    ("triangle_without_width", "piecewise-linear surrogate",
     "return net->sg_gamma * fmax(0.0, 1.0 - net->sg_beta * fabs(dv));",
     "return net->sg_gamma * fmax(0.0, 1.0 - fabs(dv));"),
    ("exponential_without_width", "exponential surrogate",
     "return net->sg_gamma * exp(-net->sg_beta * fabs(dv));", "return net->sg_gamma * exp(-fabs(dv));"),
    ("membrane_decay_from_tau_out", "exact integration of eq. lif_update",
     "p->alpha = exp(-net->dt / net->tau_m);", "p->alpha = exp(-net->dt / net->tau_out);"),
    ("adaptation_decay_from_tau_m", "exact integration of eq. spike-threshold-adaptation",
     "p->rho = exp(-net->dt / net->tau_a);", "p->rho = exp(-net->dt / net->tau_m);"),
    ("no_filter_keeps_kappa", "Results, \"Eligibility trace filter decoupled from output time constant\"",
     "net->etrace_filter == 2 ? 0.0 : p->kappa;", "net->etrace_filter == 2 ? p->kappa : p->kappa;"),
    ("refractory_steps_truncated", "refractory period in steps",
     "p->n_ref = (int)lround(net->t_ref / net->dt);", "p->n_ref = (int)(net->t_ref / net->dt) - 1;"),
    ("recurrent_spike_seen_a_step_late", "a spike of step s reaches a delay-D synapse at s + D",
     "return (s >= 1 && s <= sp->T) ? sp->zrec[(long)s * sp->J + src] : 0;",
     "return (s >= 2 && s <= sp->T) ? sp->zrec[(long)(s - 1) * sp->J + src] : 0;"),
    ("input_spike_steps_shifted", "input emission steps in [0, T-1]",
     "    sp->zin[(long)s * sp->I + i] = 1;", "    if (s + 1 < (unsigned)sp->T) sp->zin[(long)(s + 1) * sp->I + i] = 1;"),
    ("input_delay_shifted", "eq. lif_update with transmission delays",
     "if (spiked(sp, s->kind, s->src, t - s->delay))",
     "if (spiked(sp, s->kind, s->src, t - s->delay + (s->delay > 1)))"),
    # eligibility (eq. eligibility-vector-substituted, eq. filtered-eligibility-trace)
    ("eps_a_decay_psi_now", "eq. eligibility-vector-substituted",
     "const double ea_new = psi_prev * *ev + (p->rho - psi_prev * beta) * *ea;",
     "const double ea_new = psi_prev * *ev + (p->rho - psi_now * beta) * *ea;"),
    ("eps_a_input_psi_now", "eq. eligibility-vector-substituted",
     "const double ea_new = psi_prev * *ev + (p->rho - psi_prev * beta) * *ea;",
     "const double ea_new = psi_now * *ev + (p->rho - psi_prev * beta) * *ea;"),
    ("eligibility_sign", "eligibility trace",
     "const double e = psi_now * (ev_new - beta * ea_new);", "const double e = psi_now * (ev_new + beta * ea_new);"),
    ("eligibility_psi_prev", "eligibility trace",
     "const double e = psi_now * (ev_new - beta * ea_new);", "const double e = psi_prev * (ev_new - beta * ea_new);"),
    ("eps_v_with_kappa", "eq. eligibility-vector-substituted",
     "const double ev_new = (net->reset_mode == 1 && zprev != 0.0 ? 0.0 : p->alpha) * *ev + x;",
     "const double ev_new = (net->reset_mode == 1 && zprev != 0.0 ? 0.0 : p->kappa) * *ev + x;"),
    ("eps_v_ignores_full_reset", "full reset",
     "const double ev_new = (net->reset_mode == 1 && zprev != 0.0 ? 0.0 : p->alpha) * *ev + x;",
     "const double ev_new = p->alpha * *ev + x;"),
    ("decoupled_filter_ignored", "Results, \"Eligibility trace filter decoupled from output time constant\"",
     "*eb = p->kappa_e * *eb + e;", "*eb = p->kappa * *eb + e;"),
    # readout, error and loss (Methods, "Loss function")
    ("readout_leak_scaled", "eq. leaky_integrator",
     "y[k] = p->kappa * y[k] + s;", "y[k] = p->kappa * y[k] + (1.0 - p->kappa) * s;"),
    ("readout_delay_shifted", "eq. leaky_integrator_with_delay",
     "if (t - net->d_out >= 1 && sp->zrec[(long)(t - net->d_out) * J + j]) s = s + net->w_out[(long)k * J + j];",
     "if (t - net->d_out >= 1 && sp->zrec[(long)(t - net->d_out + (net->d_out > 1)) * J + j]) "
     "s = s + net->w_out[(long)k * J + j];"),
    ("mse_without_half", "eq. mean-squared-error",
     "if (win) *loss += 0.5 * d * d;", "if (win) *loss += d * d;"),
    ("mse_error_outside_window", "learning window",
     "E[k] = win ? d : 0.0;", "E[k] = d;"),
    ("cross_entropy_without_max", "eq. cross-entropy-loss",
     "if (win) *loss += -(y[label] - mx - log(se));", "if (win) *loss += -(y[label] - log(se));"),
    ("softmax_error_outside_window", "learning window",
     "E[k] = win ? pi - (k == label ? 1.0 : 0.0) : 0.0;", "E[k] = win ? pi - (k == label ? 1.0 : 0.0) : pi;"),
    ("temporal_mse_scale", "eq. temporal-mse",
     "E[k] = win ? 2.0 / K * d : 0.0;", "E[k] = win ? 1.0 / K * d : 0.0;"),
    ("learning_signal_from_w_out", "eq. final-gradient (B, not W^out)",
     "for (int k = 0; k < K; ++k) Ls = Ls + net->fb[(long)j * K + k] * E[k];\n      L_h",
     "for (int k = 0; k < K; ++k) Ls = Ls + net->w_out[(long)k * J + j] * E[k];\n      L_h"),
    # time-driven gradient (Alg. 1) and the delays (Supplementary, "Generalized delays")
    ("time_driven_fifo_not_delayed", "eq. eprop-approx-final-expanded-subs-rewritten",
     "*SYN_G(q) += Lon * L_h[(long)t * J + j] * fifo_eb[q * (dq + 1) + (t - dq) % (dq + 1)];",
     "*SYN_G(q) += Lon * L_h[(long)t * J + j] * fifo_eb[q * (dq + 1) + t % (dq + 1)];"),
    ("time_driven_ignores_d_ls", "eq. eprop-learning-signal-delay",
     "const double Lon = t <= T - net->d_ls ? 1.0 : 0.0;", "const double Lon = 1.0;"),
    ("time_driven_output_trace_lagged", "eq. eprop-output-new-subs-rewritten",
     "zb[j] = p.kappa * zb[j] + (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);",
     "zb[j] = p.kappa * zb[j] + (sp.zrec[(long)(t - 1) * J + j] ? 1.0 : 0.0);"),
    # event-driven gradient (Algs. 4 and 5)
    ("event_driven_ignores_d_ls", "eq. eprop-learning-signal-delay",
     "if (u + dq <= T - net->d_ls) *SYN_G(q) += L_h[(long)(u + dq) * J + j] * ebq;",
     "if (u + dq <= T) *SYN_G(q) += L_h[(long)(u + dq) * J + j] * ebq;"),
    ("event_driven_regulariser_window", "Methods, \"Firing rate regularization\", with delay d",
     "if (u <= T - dq) es += e;", "es += e;"),
    ("event_driven_output_alpha", "eq. eprop-output-new-subs-rewritten",
     "zbj = p.kappa * zbj + (u == seg ? 1.0 : 0.0);", "zbj = p.alpha * zbj + (u == seg ? 1.0 : 0.0);"),
    # firing-rate regularisation (Methods, "Firing rate regularization"; eq. ema-rate)
    ("regulariser_not_over_T", "Methods, \"Firing rate regularization\"",
     "creg[j] = net->c_reg / T * (f - net->f_target);", "creg[j] = net->c_reg * (f - net->f_target);"),
    ("regulariser_loss_without_half", "Methods, \"Firing rate regularization\"",
     "loss += 0.5 * net->c_reg * (f - net->f_target) * (f - net->f_target);",
     "loss += net->c_reg * (f - net->f_target) * (f - net->f_target);"),
    ("moving_rate_unnormalised", "eq. ema-rate",
     "f_h[(long)t * J + j] = p.beta_f * f_h[(long)(t - 1) * J + j] + (1.0 - p.beta_f) * z;\n      if (trace)",
     "f_h[(long)t * J + j] = p.beta_f * f_h[(long)(t - 1) * J + j] + z;\n      if (trace)"),
    ("moving_regulariser_window", "eq. ema-gradient with delay d",
     "if (t <= T - dq) *SYN_G(q) += net->c_reg * (f_h[(long)t * J + j] - net->f_target) * gh[q];",
     "*SYN_G(q) += net->c_reg * (f_h[(long)t * J + j] - net->f_target) * gh[q];"),
    # per-spike updates (Results, "Weight updates with every spike")
    ("online_cutoff_one_late", "inter-spike cutoff",
     "if (cutoff > 0 && (st->last == 0 || s - st->last >= cutoff)) {",
     "if (cutoff > 0 && (st->last == 0 || s - st->last > cutoff)) {"),
    ("online_transmits_old_weight", "update first, then transmit",
     "        *w = *w - eta * g;\n", "        I_t = I_t + *w;\n        *w = *w - eta * g;\n        I_t = I_t - *w;\n"),
    ("online_signal_without_readout_delay", "Alg. 4 with the readout delay d",
     "g += L_h[(long)(s + net->d_out) * J + j] * st->eb;", "g += L_h[(long)s * J + j] * st->eb;"),
    ("online_readout_trace_alpha", "eq. eprop-output-new-subs-rewritten",
     "*zb = p->kappa * *zb + (x ? 1.0 : 0.0);", "*zb = p->alpha * *zb + (x ? 1.0 : 0.0);"),
    ("online_flush_stops_one_early", "flush after the last step",
     "online_walk_out(net, &p, &sp, j, &zbo[j], &r_done[j], &zlast[j], T - d, cutoff, E_h, gk);",
     "online_walk_out(net, &p, &sp, j, &zbo[j], &r_done[j], &zlast[j], T - d - 1, cutoff, E_h, gk);"),
    ("online_cutoff_keeps_traces", "inter-spike cutoff",
     "      st->ev = st->ea = st->eb = st->gh = 0.0;\n", "      st->eb = st->gh = 0.0;\n"),
    ("online_lag_one_short", "the most recent learning signal",
     "const int d = net->d_out, lag = 1 + net->d_ls + net->d_out;",
     "const int d = net->d_out, lag = net->d_ls + net->d_out;"),
    # the brute-force and forward-mode checkers (dual numbers, eq. summation-future)
    ("dual_drops_threshold_derivative", "eq. pseudo-derivative through the adaptive threshold",
     "dz[(long)t * J + j] = psi * (v[j].d - A.d);", "dz[(long)t * J + j] = psi * v[j].d;"),
    ("dual_reset_not_stopped", "e-prop's reset term without a gradient",
     "dual reset = dstop((dual){zprev.x * A.x, 0.0});", "dual reset = dmul_c(zprev.x, A);"),
    ("bruteforce_future_filter_lag", "eq. summation-future",
     "fut += E_rec[(long)(t - 1) * K + k] * pow(p.kappa_e, t - d - tp);",
     "fut += E_rec[(long)(t - 1) * K + k] * pow(p.kappa_e, t - tp);"),
    ("forward_mode_readout_delay", "eq. leaky_integrator_with_delay",
     "for (int j = 0; j < J; ++j) s += net->w_out[(long)k * J + j] * dz[(long)(t - net->d_out) * J + j];",
     "for (int j = 0; j < J; ++j) s += net->w_out[(long)k * J + j] * dz[(long)t * J + j];"),
    # the sampled teacher-forced path
    ("sampled_learning_signal_lag", "eq. eprop-approx-final-expanded-subs-rewritten",
     "if (t + net->d_out <= T - net->d_ls) g += L_h[t + net->d_out] * eb;",
     "if (t + net->d_out <= T - net->d_ls) g += L_h[t] * eb;"),
    ("sampled_regulariser_over_T_twice", "Methods, \"Firing rate regularization\"",
     "const double creg = net->reg_mode == 0 ? net->c_reg / T * (nz / T - net->f_target) : 0.0;",
     "const double creg = net->reg_mode == 0 ? net->c_reg / T * (nz / T / T - net->f_target) : 0.0;"),
    ("sampled_moving_rate_unnormalised", "eq. ema-rate",
     "f = p.beta_f * f + (1.0 - p.beta_f) * (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);\n          gh",
     "f = p.beta_f * f + (sp.zrec[(long)t * J + j] ? 1.0 : 0.0);\n          gh"),
    ("sampled_loss_regulariser_without_half", "eq. sma-loss",
     "if (net->reg_mode == 1) loss += 0.5 * net->c_reg * sf;", "if (net->reg_mode == 1) loss += net->c_reg * sf;"),
    ("bruteforce_moving_filter_unnormalised", "eq. ema-gradient",
     "for (int s1 = 1; s1 <= s2; ++s1) G += (1.0 - p.beta_f) * pow(p.beta_f, s2 - s1) * dz[(long)s1 * J + sd.tgt];",
     "for (int s1 = 1; s1 <= s2; ++s1) G += pow(p.beta_f, s2 - s1) * dz[(long)s1 * J + sd.tgt];"),
    # optimiser (Methods, "Optimization")
    ("adam_without_second_moment_correction", "eq. eta-adam-fast",
     "const double eta_t = eta * sqrt(1.0 - pow(beta2, (double)step)) / (1.0 - pow(beta1, (double)step));",
     "const double eta_t = eta / (1.0 - pow(beta1, (double)step));"),
    ("adam_epsilon_inside_root", "eq. delta-w-adam-fast",
     "w[i] = w[i] - eta_t * m[i] / (sqrt(v[i]) + eps_hat);", "w[i] = w[i] - eta_t * m[i] / sqrt(v[i] + eps_hat);"),
    ("sum_instead_of_mean", "eq. gradient-descent on the mini-batch mean",
     "const double G = g_sum[i] / n_trials;", "const double G = g_sum[i];"),
    # class prediction (arg max of the window-summed softmax or readout)
    ("prediction_ignores_window_ce", "prediction from the learning window (eq. softmax)",
     "if (win) psum[k] += pi;", "psum[k] += pi;"),
    ("prediction_ignores_window_tmse", "prediction from the learning window (eq. temporal-mse)",
     "if (win) {\n        *loss += d * d / K;\n        psum[k] += y[k];\n      }",
     "if (win) *loss += d * d / K;\n      psum[k] += y[k];"),
    ("prediction_ce_sums_readout", "cross-entropy predicts from the softmax output",
     "if (win) psum[k] += pi;", "if (win) psum[k] += y[k];"),
    ("prediction_arg_min", "the predicted class is the arg max",
     "if (psum[k] > psum[best]) best = k;\n    *pred", "if (psum[k] < psum[best]) best = k;\n    *pred"),
    ("prediction_last_of_ties", "ties go to the lowest index",
     "if (psum[k] > psum[best]) best = k;\n    *pred", "if (psum[k] >= psum[best]) best = k;\n    *pred"),
    # running error bounds for checking FP32 evaluations (Higham, sec. 3.3)
    ("fp32_bound_membrane_without_memory", "running error of v = alpha v + I - z A",
     "mu_v = p.alpha * mu_v + 2.0 * fabs(p.alpha * v_prev)", "mu_v = 2.0 * fabs(p.alpha * v_prev)"),
    ("fp32_bound_adaptation_without_memory", "running error of a = rho a + z",
     "mu_a = p.rho * mu_a + 2.0 * fabs(p.rho * a_prev) + fabs(a);", "mu_a = 2.0 * fabs(p.rho * a_prev) + fabs(a);"),
    ("fp32_bound_quantum_ignored", "weights rounded by a fixed-point accumulator",
     "const double mu_I = fabs(I_t) + n_arr * quantum / u;", "const double mu_I = fabs(I_t);"),
    ("fp32_bound_given_psi_shifted", "the archived psi history, row t-1 is step t",
     "psi_h[t] = psi_given ? psi_given[(long)(t - 1) * J + j] : psi;",
     "psi_h[t] = psi_given ? psi_given[(long)(t > 1 ? t - 2 : 0) * J + j] : psi;"),
    ("fp32_bound_signed_learning_signal", "absolute term sum of the gradient",
     "La = La + fabs(net->fb[(long)j * K + k] * E_h[(long)t * K + k]);",
     "La = La + net->fb[(long)j * K + k] * E_h[(long)t * K + k];"),
]


def _copy_tree(dst):
    """The oracle, the pins and the input generators they use; nothing built."""
    skip = shutil.ignore_patterns("__pycache__", ".pytest_cache", "*.so", "*.so.tmp*")
    for part in ("oracle", "tests", "paper_2511_21674_amd"):
        shutil.copytree(os.path.join(ROOT, part), os.path.join(dst, part), ignore=skip)


def run_one(entry, base):
    """Runs the pins on a copy of the oracle with one mistake planted (none
    for the control entry, whose pins must pass)."""
    name, _, good, bad = entry
    work = os.path.join(base, name)
    _copy_tree(work)
    path = os.path.join(work, SRC)
    src = open(path).read()
    if good is not None:
        if src.count(good) != 1:
            return name, "NOT FOUND (the oracle changed; update this entry)"
        with open(path, "w") as f:
            f.write(src.replace(good, bad))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=work,
                       capture_output=True, text=True, env=env)
    if r.returncode:
        return name, "BUILD FAILED " + r.stderr[-200:]
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle.py", "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=work, capture_output=True, text=True, env=env)
    shutil.rmtree(work, ignore_errors=True)
    if r.returncode == 0:
        return name, "SURVIVED"
    first = next((ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")), "failed")
    return name, "caught by " + first.split(" - ")[0].replace("FAILED ", "")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=4)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    todo = [m for m in MUTATIONS if not args.names or m[0] in args.names]
    base = tempfile.mkdtemp(prefix="oracle_mut_")
    bad = 0
    try:
        # control: the copied pins pass on the unchanged oracle
        name, verdict = run_one(("control", "", None, None), base)
        if verdict != "SURVIVED":
            print(f"the pins fail on the unchanged oracle ({verdict}); nothing to check", flush=True)
            return 2
        with ThreadPoolExecutor(max_workers=max(1, args.j)) as ex:
            for name, verdict in ex.map(lambda m: run_one(m, base), todo):
                bad += not verdict.startswith("caught")
                print(f"{name:42s} {verdict}", flush=True)
    finally:
        shutil.rmtree(base, ignore_errors=True)
    print(f"{len(todo) - bad} of {len(todo)} planted mistakes caught", flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
