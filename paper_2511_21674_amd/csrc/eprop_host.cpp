// Host side of the C ABI declared in include/eprop.h: argument validation
// (before any device work), graph construction in source- and target-major
// order, device memory, the step loop (captured once into a HIP graph per
// block of steps and replayed), the optimizer call and state read-back.
#include "eprop.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "eprop_internal.h"

static_assert(eprop::kScratchBytes == EPROP_NOALLOC_SCRATCH_BYTES, "staging array size");

using eprop::DevNet;
using eprop::Launch;
using eprop::Shapes;

namespace {
thread_local std::string g_create_error;
constexpr uint32_t kMaxIndex = (1u << 24) - 1u;


inline bool is_finite(double x) { return std::isfinite(x); }
inline uint32_t round_up(uint32_t a, uint32_t m) { return (a + m - 1) / m * m; }

// Host threads for building graphs of 10^9 synapses (at most 16).
unsigned host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return std::max(1u, std::min(h ? h : 1u, 16u));
}

// Runs f(lo, hi, t) on nt threads over consecutive ranges of [0, n) whose
// boundaries split the weight w(0..n) (a non-decreasing prefix such as a
// CSR row pointer) evenly; t is the range's rank.
template <typename W, typename F>
void parallel_ranges(uint64_t n, unsigned nt, W w, F f) {
  if (nt <= 1 || n < 2) {
    f((uint64_t)0, n, 0u);
    return;
  }
  std::vector<uint64_t> cut(nt + 1, n);
  cut[0] = 0;
  const double total = (double)w(n);
  for (unsigned t = 1; t < nt; ++t) {
    uint64_t lo = cut[t - 1], hi = n;  // first index whose prefix reaches t / nt of the total
    const double goal = total * t / nt;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if ((double)w(mid) < goal) lo = mid + 1; else hi = mid;
    }
    cut[t] = lo;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) th.emplace_back([&, t] { f(cut[t], cut[t + 1], t); });
  for (auto &x : th) x.join();
}
}  // namespace

struct eprop_network {
  eprop_config cfg{};
  uint32_t I = 0, J = 0, K = 0, NS = 0, Jp = 0, Jw = 0, Iw = 0, R = 0, Tcap = 0, Tp = 0, Bcap = 0, Ts = 0;
  uint64_t S_in = 0, S_rec = 0, S = 0;
  bool fp64 = false, gather = false, adam = false, use_graph = true;
  uint32_t n_ref = 0;
  double alpha = 0, rho = 0, kappa = 0;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  bool failed = false;
  std::string err;
  std::vector<void *> allocs;
  DevNet<float> n32{};
  DevNet<double> n64{};
  Shapes shapes{};
  std::vector<uint32_t> perm;       // target-major index -> caller's synapse index
  std::vector<uint32_t> sm2caller;  // internal source-major index -> caller's synapse index
  size_t tile_smem = 0;             // dynamic LDS of the tiled forward kernel
  bool blocked = false;             // weight update as a blocked transposition (k_apply_blk)
  bool queues = false;              // per-tile queues built (FP32 scatter; forward variant kQueueVariant)
  uint32_t q_since = 0;             // queue step tags used since the queues were last cleared
  uint64_t dl_words = 0;            // size of the delivery table (4-byte words)
  bool dl_packed = false;           // its segments packed (the line-aligned placement would exceed 2^31 words)
  // e-prop+ schedule (allocated on the first online batch)
  void *on_syn = nullptr;
  double *on_Eh = nullptr, *on_y = nullptr, *on_zbo = nullptr, *on_loss = nullptr, *on_psum = nullptr;
  uint32_t *on_rdone = nullptr, *on_zlast = nullptr, *on_off = nullptr, *on_label = nullptr;
  void *on_fh = nullptr, *on_I = nullptr, *on_L = nullptr;
  size_t cap_on_loss = 0, cap_on_psum = 0, cap_on_off = 0, cap_on_label = 0;
  uint32_t n_ach = 0;               // its blocks
  void *partial = nullptr;          // per trial-chunk synapse sums (large batches)
  void *Lbuf = nullptr;             // learning signal of the time-driven baseline (allocated on first use)
  size_t cap_Lbuf = 0;
  uint32_t trials_accum = 0;
  uint64_t adam_step = 0;
  // library-owned staging copies of host-memory batches
  uint32_t *d_T = nullptr, *d_label = nullptr;
  uint64_t *d_in_ptr = nullptr, *d_forced_ptr = nullptr;
  uint32_t *d_in_step = nullptr, *d_in_src = nullptr, *d_forced_step = nullptr, *d_forced_neuron = nullptr;
  double *d_target = nullptr;
  uint8_t *d_window = nullptr;
  size_t cap_in_step = 0, cap_in_src = 0, cap_target = 0, cap_window = 0, cap_f_step = 0, cap_f_neuron = 0;
  // host copies reused by every batch (reserved at create for max_trials)
  std::vector<uint64_t> h_in_ptr, h_f_ptr;
  std::vector<double> h_loss;
  std::vector<uint32_t> h_pred;
  // eprop_simulate_batch_noalloc: this device's static staging array
  uint8_t *scratch = nullptr;
  // step loop
  uint32_t blk = 0;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipEvent_t ev[EPROP_N_PHASES + 1] = {};
  hipEvent_t tev[2] = {};           // autotuner timing
  bool autotune_pending = false, tuned = false;
  // last batch
  uint32_t last_ntr = 0;
  std::vector<uint32_t> last_T;
};

namespace {

void set_fail(eprop_network *n, const std::string &m) { n->err = m; }

// Places a delivery-table segment of L synapses (L weights of sz bytes, then
// L uint16 ring offsets, rounded up to a multiple of sz) at byte cur or
// later: on the next kDlGrain boundary if it is longer than kDlGrain or
// would otherwise cross a boundary that it fits between (unless packed).
// Returns the end.
uint64_t dl_place(uint64_t cur, uint64_t L, uint64_t sz, uint64_t *at, bool packed) {
  const uint64_t G = eprop::kDlGrain, z = (L * (sz + 2) + sz - 1) / sz * sz;
  if (!packed && z > 0 && (z > G || cur % G + z > G)) cur = (cur + G - 1) / G * G;
  *at = cur;
  return cur + z;
}

// Message for a host-side exception caught at the ABI (allocation or thread
// creation failed); such a failure is reported as EPROP_ERR_OUT_OF_MEMORY.
std::string host_failure(const std::exception &x) {
  if (dynamic_cast<const std::bad_alloc *>(&x)) return "host allocation failed";
  return std::string("host resource failure: ") + x.what();
}

void dfree(eprop_network *n, void *p) {
  if (!p) return;
  if (n->cfg.dev_free) n->cfg.dev_free(p, n->cfg.alloc_ctx);
  else (void)hipFree(p);
}

template <typename T>
bool dalloc(eprop_network *n, T **p, size_t count) {
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  void *q = nullptr;
  if (n->cfg.dev_alloc) {
    q = n->cfg.dev_alloc(bytes, n->cfg.alloc_ctx);
    if (q && (reinterpret_cast<uintptr_t>(q) & 255u) != 0) {  // the kernels assume 256-byte alignment
      n->cfg.dev_free(q, n->cfg.alloc_ctx);
      q = nullptr;
    }
  } else if (hipMalloc(&q, bytes) != hipSuccess) {
    q = nullptr;
    (void)hipGetLastError();
  }
  *p = static_cast<T *>(q);
  if (!q) return false;
  n->allocs.push_back(q);
  return true;
}

// Grows a library-owned staging buffer; returns false on allocation failure.
template <typename T>
bool dgrow(eprop_network *n, T **p, size_t *cap, size_t count) {
  if (*p && *cap >= count) return true;
  if (*p) {
    auto it = std::find(n->allocs.begin(), n->allocs.end(), (void *)*p);
    if (it != n->allocs.end()) n->allocs.erase(it);
    dfree(n, *p);
    *p = nullptr;
  }
  const size_t want = std::max<size_t>(count, 1024);
  if (!dalloc(n, p, want)) return false;
  *cap = want;
  return true;
}

const char *hip_msg(hipError_t e) { return hipGetErrorString(e); }

eprop_status check_projection(const eprop_projection *p, uint32_t n_src, uint32_t n_tgt, uint32_t max_delay,
                              bool no_self, const char *name, std::string &msg) {
  if (!p) { msg = std::string(name) + ": NULL projection"; return EPROP_ERR_INVALID_ARGUMENT; }
  if (p->n_src != n_src || p->n_tgt != n_tgt) {
    msg = std::string(name) + ": n_src/n_tgt do not match the network sizes";
    return EPROP_ERR_INVALID_ARGUMENT;
  }
  if (!p->row_ptr) { msg = std::string(name) + ": NULL row_ptr"; return EPROP_ERR_INVALID_ARGUMENT; }
  if (p->row_ptr[0] != 0 || p->row_ptr[n_src] != p->nnz) {
    msg = std::string(name) + ": row_ptr must start at 0 and end at nnz";
    return EPROP_ERR_INVALID_ARGUMENT;
  }
  if (p->nnz > 0 && (!p->col || !p->w)) { msg = std::string(name) + ": NULL col or w"; return EPROP_ERR_INVALID_ARGUMENT; }
  for (uint32_t i = 0; i < n_src; ++i) {
    if (p->row_ptr[i] > p->row_ptr[i + 1]) {
      msg = std::string(name) + ": row_ptr decreases";
      return EPROP_ERR_INVALID_ARGUMENT;
    }
    for (uint64_t q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
      if (p->col[q] >= n_tgt) { msg = std::string(name) + ": target index out of range"; return EPROP_ERR_INVALID_ARGUMENT; }
      if (no_self && p->col[q] == i) { msg = std::string(name) + ": self-connection"; return EPROP_ERR_INVALID_ARGUMENT; }
      const uint32_t d = p->delay ? p->delay[q] : 1u;
      if (d < 1 || d > max_delay) { msg = std::string(name) + ": delay outside 1..max_delay"; return EPROP_ERR_INVALID_ARGUMENT; }
      if (!is_finite(p->w[q])) { msg = std::string(name) + ": non-finite weight"; return EPROP_ERR_INVALID_ARGUMENT; }
    }
  }
  return EPROP_OK;
}

eprop_status check_config(const eprop_config *c, std::string &msg) {
  if (!c) { msg = "NULL config"; return EPROP_ERR_INVALID_ARGUMENT; }
  if (c->abi_version != EPROP_ABI_VERSION) { msg = "ABI version mismatch"; return EPROP_ERR_UNSUPPORTED; }
  auto bad = [&](const char *m) { msg = m; return EPROP_ERR_INVALID_ARGUMENT; };
  if (c->precision != EPROP_FP32 && c->precision != EPROP_FP64) return bad("precision must be FP32 or FP64");
  if (c->n_rec < 1) return bad("n_rec must be >= 1");
  if (c->n_out < 1 || c->n_out > 64) return bad("n_out must be in 1..64");
  if ((uint64_t)c->n_in + c->n_rec > kMaxIndex) return bad("n_in + n_rec must be below 2^24");
  if (!(c->dt > 0) || !(c->tau_m > 0) || !(c->tau_out > 0) || !(c->tau_a > 0) || !is_finite(c->dt) ||
      !is_finite(c->tau_m) || !is_finite(c->tau_out) || !is_finite(c->tau_a))
    return bad("dt and time constants must be positive and finite");
  if (!is_finite(c->v_th) || !is_finite(c->beta_a) || !is_finite(c->sg_gamma) || !is_finite(c->sg_beta))
    return bad("non-finite neuron or surrogate parameter");
  // (compared before rounding: lround of a quotient beyond the long range is unspecified)
  if (!(c->t_ref >= 0) || !is_finite(c->t_ref) || !(c->t_ref / c->dt < 127.5))
    return bad("t_ref must give 0..127 refractory steps");
  if (c->surrogate != EPROP_SG_PIECEWISE_LINEAR && c->surrogate != EPROP_SG_EXPONENTIAL) return bad("unknown surrogate");
  if (c->loss != EPROP_LOSS_MSE && c->loss != EPROP_LOSS_SOFTMAX_CE && c->loss != EPROP_LOSS_TEMPORAL_MSE)
    return bad("unknown loss");
  if (c->optimizer != EPROP_OPT_GD && c->optimizer != EPROP_OPT_ADAM) return bad("unknown optimizer");
  if (!is_finite(c->eta)) return bad("non-finite learning rate");
  if (c->optimizer == EPROP_OPT_ADAM &&
      (!(c->adam_beta1 >= 0 && c->adam_beta1 < 1) || !(c->adam_beta2 >= 0 && c->adam_beta2 < 1) ||
       !(c->adam_eps_hat > 0) || !is_finite(c->adam_eps_hat)))
    return bad("Adam parameters out of range");
  if (c->max_delay < 1 || c->max_delay > 255) return bad("max_delay must be in 1..255");
  if (c->max_trials < 1) return bad("max_trials must be >= 1");
  if (c->max_steps < 1 || c->max_steps > 65535) return bad("max_steps must be in 1..65535");
  if (c->delivery < EPROP_DELIVERY_AUTO || c->delivery > EPROP_DELIVERY_GATHER) return bad("unknown delivery");
  if (c->flags & ~(uint32_t)(EPROP_FLAG_NO_GRAPH | EPROP_DETERMINISTIC | EPROP_SHARED_WEIGHTS | EPROP_AUTOTUNE |
                             EPROP_SCATTER_LOOKUP | EPROP_SCATTER_QUEUES))
    return bad("unknown config flag");
  if ((c->flags & EPROP_SCATTER_LOOKUP) && (c->flags & EPROP_SCATTER_QUEUES))
    return bad("EPROP_SCATTER_LOOKUP and EPROP_SCATTER_QUEUES exclude each other");
  if ((c->flags & EPROP_DETERMINISTIC) && c->precision == EPROP_FP64 && c->delivery == EPROP_DELIVERY_SCATTER)
    return bad("FP64 scatter delivery is not deterministic; use gather or AUTO");
  if ((c->dev_alloc == nullptr) != (c->dev_free == nullptr)) return bad("dev_alloc and dev_free go together");
  if (c->d_out > 65535 || c->d_ls > 65535) return bad("d_out and d_ls must be in 0..65535");
  if (!(c->c_reg >= 0) || !is_finite(c->c_reg)) return bad("c_reg must be finite and >= 0");
  if (!(c->f_target >= 0) || !is_finite(c->f_target)) return bad("f_target must be finite and >= 0");
  if (c->reset_mode != EPROP_RESET_SUBTRACT && c->reset_mode != EPROP_RESET_TO_VALUE) return bad("unknown reset_mode");
  if (!is_finite(c->v_reset)) return bad("non-finite v_reset");
  if (c->etrace_filter < EPROP_ETRACE_COUPLED || c->etrace_filter > EPROP_ETRACE_NONE)
    return bad("unknown etrace_filter");
  if (c->etrace_filter == EPROP_ETRACE_DECOUPLED && (!(c->tau_e > 0) || !is_finite(c->tau_e)))
    return bad("tau_e must be finite and > 0 for the decoupled eligibility filter");
  if (c->reg_mode != EPROP_REG_STATIC && c->reg_mode != EPROP_REG_MOVING_AVERAGE) return bad("unknown reg_mode");
  if (c->reg_mode == EPROP_REG_MOVING_AVERAGE && (!(c->reg_tau > 0) || !is_finite(c->reg_tau)))
    return bad("reg_tau must be finite and > 0 for the moving-average regulariser");
  if (c->history_steps != 0 && c->history_steps < c->max_steps) {
    msg = "the history covers whole trials: history_steps must be 0 or >= max_steps";
    return EPROP_ERR_UNSUPPORTED;
  }
  return EPROP_OK;
}

// Fills a DevNet's pointers and constants from the network's allocations.
template <typename real>
bool alloc_state(eprop_network *n, DevNet<real> &d) {
  const size_t B = n->Bcap, T1 = (size_t)n->Tcap + 1, T2 = (size_t)n->Tcap + 2;
  d.I = n->I; d.J = n->J; d.K = n->K; d.NS = n->NS; d.Jp = n->Jp; d.Jw = n->Jw; d.Iw = n->Iw;
  d.R = n->R; d.Tcap = n->Tcap; d.Tp = n->Tp; d.Bcap = n->Bcap; d.Ts = n->Ts;
  d.Lc = round_up(n->Tcap, 8);
  d.spk_stride = (uint64_t)n->NS * d.Lc;
  d.S = n->S;
  d.n_ref = n->n_ref;
  d.surrogate = n->cfg.surrogate;
  d.loss = n->cfg.loss;
  d.alpha = (real)n->alpha; d.rho = (real)n->rho; d.v_th = (real)n->cfg.v_th;
  d.sg_gamma = (real)n->cfg.sg_gamma; d.sg_beta = (real)n->cfg.sg_beta;
  d.alpha_d = n->alpha; d.rho_d = n->rho; d.kappa_d = n->kappa;
  d.d_out = n->cfg.d_out; d.d_ls = n->cfg.d_ls;
  d.c_reg = n->cfg.c_reg;
  d.f_target = n->cfg.f_target * n->cfg.dt / 1000.0;
  d.reset_mode = n->cfg.reset_mode;
  d.v_reset = (real)n->cfg.v_reset;
  d.kappa_e_d = n->cfg.etrace_filter == EPROP_ETRACE_DECOUPLED ? std::exp(-n->cfg.dt / n->cfg.tau_e)
                : n->cfg.etrace_filter == EPROP_ETRACE_NONE ? 0.0 : n->kappa;
  d.reg_mode = n->cfg.c_reg != 0.0 ? n->cfg.reg_mode : EPROP_REG_STATIC;
  d.beta_f = n->cfg.reg_mode == EPROP_REG_MOVING_AVERAGE ? std::exp(-n->cfg.dt / n->cfg.reg_tau) : 0.0;
  uint32_t *p32;
  real *pr;
  bool ok = true;
  d.TS = n->n32.TS ? n->n32.TS : n->n64.TS;
  d.KT = n->n32.KT ? n->n32.KT : n->n64.KT;
  d.ring_bytes = n->n32.ring_bytes ? n->n32.ring_bytes : n->n64.ring_bytes;
  ok &= dalloc(n, &p32, n->NS + 1); d.sm_ptr = p32;
  if (!n->gather) {
    ok &= dalloc(n, &p32, (size_t)n->NS * (d.KT + 1)); d.tseg = p32;
  }
  ok &= dalloc(n, &d.nspk, B * T1);
  ok &= dalloc(n, &p32, n->J + 1); d.tm_ptr = p32;
  ok &= dalloc(n, &p32, n->S); d.tm_syn = p32;
  if (!n->gather) {
    ok &= dalloc(n, &p32, n->S); d.tm_dpos = p32;
  }
  ok &= dalloc(n, &p32, (size_t)n->NS * n->R); d.outdeg = p32;
  if (n->blocked) ok &= dalloc(n, &d.tsum, n->Jp);
  else ok &= dalloc(n, &d.tm_w, n->S);
  ok &= dalloc(n, &d.gs, n->S);
  ok &= dalloc(n, &d.gc, n->S);
  if (n->adam) {
    ok &= dalloc(n, &d.adam_m, n->S);
    ok &= dalloc(n, &d.adam_v, n->S);
  }
  ok &= dalloc(n, &pr, n->Jp); d.beta_j = pr;
  const size_t KJ = (size_t)n->K * n->Jp;
  ok &= dalloc(n, &d.w_out, KJ);
  ok &= dalloc(n, &d.fb, KJ);
  ok &= dalloc(n, &d.gos, KJ);
  ok &= dalloc(n, &d.goc, KJ);
  if (n->adam) {
    ok &= dalloc(n, &d.adam_mo, KJ);
    ok &= dalloc(n, &d.adam_vo, KJ);
  }
  ok &= dalloc(n, &d.gout_b, B * KJ);
  ok &= dalloc(n, &d.v, B * n->Jp);
  ok &= dalloc(n, &d.a, B * n->Jp);
  ok &= dalloc(n, &d.nst, B * n->Jp);
  {
    uint8_t *rp = nullptr;
    ok &= dalloc(n, &rp, B * n->R * n->Jp * d.ring_bytes);
    d.ring = rp;
  }
  ok &= dalloc(n, &d.l1max, 1);
  ok &= dalloc(n, &d.psi, B * T1 * n->Jp);
  ok &= dalloc(n, &d.phi, B * n->Jp * n->Tp);
  ok &= dalloc(n, &d.rec_bits, B * T1 * n->Jw);
  ok &= dalloc(n, &d.in_bits, B * n->Tcap * n->Iw);
  ok &= dalloc(n, &d.forced_bits, B * T1 * n->Jw);   // teacher-forced spikes (no allocation in a batch call)
  ok &= dalloc(n, &d.spk_cnt, B * n->NS);
  ok &= dalloc(n, &d.spk_t, B * d.spk_stride);
  ok &= dalloc(n, &d.pub_list, B * 2 * n->Jp);
  ok &= dalloc(n, &d.pub_cnt, B * 2 * (size_t)d.KT);
  ok &= dalloc(n, &d.in_step_ptr, B * T1);
  ok &= dalloc(n, &d.ysum, B * T2 * n->K);
  ok &= dalloc(n, &d.y, B * T2 * n->K);
  ok &= dalloc(n, &d.err, B * T2 * n->K);
  ok &= dalloc(n, &d.ebar, B * T2 * n->K);
  if (n->cfg.d_ls || n->cfg.etrace_filter != EPROP_ETRACE_COUPLED) ok &= dalloc(n, &d.ebo, B * T2 * n->K);
  else d.ebo = d.ebar;
  ok &= dalloc(n, &d.loss_out, B);
  ok &= dalloc(n, &d.pred_out, B);
  ok &= dalloc(n, &d.ctl, 64);
  ok &= dalloc(n, &d.cnt, eprop::CNT_WORDS);
  ok &= dalloc(n, &d.evcnt, 64);
  const uint32_t nchunk_max = (n->Bcap + n->shapes.ginst - 1) / n->shapes.ginst;
  {
    // worst case: every record has a header and a partly used last block,
    // rounded up to its size class (under twice its size), the class regions
    // start on lines, and slack follows for the synapse kernel's prefetch
    const size_t recs = (size_t)nchunk_max * n->NS;
    d.pk_cap = 3 * (2 * recs + (B * n->NS * (size_t)d.Lc + 7) / 8) + 40;
    ok &= d.pk_cap < 0xFFFFFFF0ull;
    ok &= dalloc(n, &d.pk_off, recs + 1);
    ok &= dalloc(n, &d.pk_bsum, ((recs + eprop::kScanItems - 1) / eprop::kScanItems + 1) * 4);
    ok &= dalloc(n, &d.pk, d.pk_cap * 8);
  }
  if (nchunk_max > 1) {
    real *part = nullptr;
    ok &= dalloc(n, &part, (size_t)nchunk_max * n->S);
    n->partial = part;
  }
  return ok;
}

// Uploads graph, weights and optimiser state (host arrays in double).
// Tables and buffers of the per-tile queues: every recurrent neuron's
// non-empty tile segments (q_nzp, q_nz), then, from q_nz[q_in], one entry
// per input i and tile k: the segment of i into tile (k - i) mod KT, which
// tile k copies when i spikes (so an input spike's segments are spread over
// all tiles); and the regions of the event buffers, one per (source tile,
// target tile) pair, sized by the synapses the source tile copies into the
// target tile (those of its own neurons and its input segments), ordered by
// target tile, then source tile (q_src row k: the starts of tile k's
// regions as a source; q_dst row k: those of the regions into tile k).  The
// buffers start cleared.
template <typename real>
hipError_t upload_queues(eprop_network *n, DevNet<real> &d, const std::vector<uint32_t> &tseg,
                         const std::vector<uint2> &dsegh) {
  const uint32_t KT = d.KT, TS = d.TS, J = n->J, I = n->I;
  const unsigned nt = n->S >= (1u << 22) ? host_threads() : 1u;
  auto L_of = [&](uint64_t src, uint32_t k) {
    return tseg[src * (KT + 1) + k + 1] - tseg[src * (KT + 1) + k];
  };
  std::vector<uint32_t> nzp((size_t)J + 1, 0u);
  auto flat = [](uint64_t i) { return i; };
  parallel_ranges(J, nt, flat, [&](uint64_t lo, uint64_t hi, unsigned) {
    for (uint64_t j = lo; j < hi; ++j) {
      uint32_t c = 0;
      for (uint32_t k = 0; k < KT; ++k) c += L_of(I + j, k) > 0;
      nzp[j + 1] = c;
    }
  });
  for (uint32_t j = 0; j < J; ++j) nzp[j + 1] += nzp[j];
  const uint64_t q_in = nzp[J];
  if (q_in + (uint64_t)I * KT >= (1ull << 32)) return hipErrorInvalidValue;
  std::vector<uint2> nz(std::max<uint64_t>(q_in + (uint64_t)I * KT, 1), make_uint2(0u, 0u));
  std::vector<uint64_t> rsz((size_t)KT * KT, 0);
  parallel_ranges(KT, std::min<unsigned>(nt, KT), flat, [&](uint64_t k0, uint64_t k1, unsigned) {
    for (uint64_t ks = k0; ks < k1; ++ks) {
      for (uint64_t j = ks * TS; j < std::min<uint64_t>(J, (ks + 1) * TS); ++j) {
        uint32_t at = nzp[j];
        for (uint32_t kd = 0; kd < KT; ++kd) {
          const uint32_t L = L_of(I + j, kd);
          if (L == 0) continue;
          nz[at++] = make_uint2(dsegh[(I + j) * KT + eprop::tile_rank(kd, KT)].x, L | kd << 16);
          rsz[ks * KT + kd] += L;
        }
      }
      for (uint64_t i = 0; i < I; ++i) {  // input i's segment into tile (ks - i) mod KT
        const uint32_t kd = (uint32_t)((ks + KT - i % KT) % KT), L = L_of(i, kd);
        nz[q_in + i * KT + ks] = make_uint2(L ? dsegh[i * KT + eprop::tile_rank(kd, KT)].x : 0u, L | kd << 16);
        rsz[ks * KT + kd] += L;
      }
    }
  });
  std::vector<uint32_t> qsrc((size_t)KT * KT), qdst((size_t)KT * KT);
  uint64_t acc = 0;
  for (uint32_t kd = 0; kd < KT; ++kd)
    for (uint32_t ks = 0; ks < KT; ++ks) {
      qdst[(size_t)kd * KT + ks] = qsrc[(size_t)ks * KT + kd] = (uint32_t)acc;
      acc += rsz[(size_t)ks * KT + kd];
    }
  if (acc != n->S) return hipErrorInvalidValue;  // every synapse in exactly one region
  d.q_len = (uint32_t)std::max<uint64_t>(acc, 1);
  uint32_t *p_nzp = nullptr, *p_src = nullptr, *p_dst = nullptr;
  uint2 *p_nz = nullptr;
  uint64_t *p_ev = nullptr, *p_hdr = nullptr;
  const size_t kt2 = (size_t)KT * KT, nev = (size_t)n->Bcap * 2 * d.q_len, nhdr = (size_t)n->Bcap * 2 * kt2;
  if (!dalloc(n, &p_nzp, nzp.size()) || !dalloc(n, &p_nz, nz.size()) || !dalloc(n, &p_src, kt2) ||
      !dalloc(n, &p_dst, kt2) || !dalloc(n, &p_ev, nev) || !dalloc(n, &p_hdr, nhdr))
    return hipErrorOutOfMemory;
  hipError_t e = hipMemcpy(p_nzp, nzp.data(), nzp.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p_nz, nz.data(), nz.size() * sizeof(uint2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p_src, qsrc.data(), kt2 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p_dst, qdst.data(), kt2 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p_ev, 0, nev * 8);
  if (e == hipSuccess) e = hipMemset(p_hdr, 0, nhdr * 8);
  d.q_nzp = p_nzp;
  d.q_nz = p_nz;
  d.q_in = (uint32_t)q_in;
  d.q_src = p_src;
  d.q_dst = p_dst;
  d.q_ev = p_ev;
  d.q_hdr = p_hdr;
  n->q_since = 0;
  return e;
}

template <typename real>
hipError_t upload(eprop_network *n, DevNet<real> &d, const std::vector<uint32_t> &sm_ptr,
                  const std::vector<uint32_t> &tseg,
                  const std::vector<uint32_t> &sm_syn, const std::vector<double> &sm_w,
                  const std::vector<uint32_t> &tm_ptr, const std::vector<uint32_t> &tm_syn,
                  const std::vector<uint32_t> &tm_perm, const std::vector<double> &tm_w,
                  const std::vector<double> &beta, const double *w_out, const double *fb,
                  const eprop_optimizer_state *opt) {
  hipError_t e = hipSuccess;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  const unsigned nt = n->S >= (1u << 22) ? host_threads() : 1u;
  auto flat = [](uint64_t i) { return i; };
  auto conv = [&](const std::vector<double> &v) {
    std::vector<real> o(v.size());
    parallel_ranges(v.size(), nt, flat, [&](uint64_t lo, uint64_t hi, unsigned) {
      for (uint64_t i = lo; i < hi; ++i) o[i] = (real)v[i];
    });
    return o;
  };
  cp((void *)d.sm_ptr, sm_ptr.data(), sm_ptr.size() * 4);
  if (!n->gather) {
    cp((void *)d.tseg, tseg.data(), tseg.size() * 4);
    // delivery table: each source's part starts on a kDlGrain boundary (so
    // that the parts can be laid out independently); inside it, the
    // segments of the tiles in tile_rank order, each placed by dl_place.
    // The kernels index the ring offsets in uint16 units with 32-bit
    // integers, so the table holds under 2^31 words; where the line-aligned
    // placement would not fit that (its padding costs up to a third at
    // segments of 40 synapses, as in the paper's scaling network), the
    // segments are packed instead.
    const uint32_t KT = d.KT, TS = d.TS;
    const uint64_t NS = n->NS;
    std::vector<uint32_t> by_rank(KT);  // the tile at each place
    for (uint32_t k = 0; k < KT; ++k) by_rank[eprop::tile_rank(k, KT)] = k;
    auto src_weight = [&](uint64_t src) { return (uint64_t)sm_ptr[src]; };
    std::vector<uint64_t> part(NS + 1, 0);
    uint64_t total = 0;
    bool packed = false;
    for (int pass = 0; pass < 2; ++pass) {
      packed = pass == 1;
      parallel_ranges(NS, nt, src_weight, [&](uint64_t s0, uint64_t s1, unsigned) {
        for (uint64_t src = s0; src < s1; ++src) {
          uint64_t cur = 0, at = 0;
          for (uint32_t r = 0; r < KT; ++r) {
            const uint32_t k = by_rank[r];
            cur = dl_place(cur, tseg[src * (KT + 1) + k + 1] - tseg[src * (KT + 1) + k], sizeof(real), &at, packed);
          }
          part[src] = (cur + eprop::kDlGrain - 1) / eprop::kDlGrain * eprop::kDlGrain;
        }
      });
      total = 0;
      for (uint64_t src = 0; src < NS; ++src) {
        const uint64_t b = part[src];
        part[src] = total;
        total += b;
      }
      part[NS] = total;
      if (total / 4 < (1ull << 31)) break;
    }
    if (total / 4 >= (1ull << 31)) {
      g_create_error = "the delivery table needs " + std::to_string(total >> 20) +
                       " MiB, more than the 8 GiB its 32-bit uint16 indices address";
      return hipErrorNotSupported;
    }
    n->dl_packed = packed;
    n->dl_words = std::max<uint64_t>(total / 4, 1);
    std::vector<uint32_t> dlh(n->dl_words, 0u), dpos(n->S, 0u);
    std::vector<uint2> dsegh((size_t)NS * KT);
    parallel_ranges(NS, nt, src_weight, [&](uint64_t s0, uint64_t s1, unsigned) {
      for (uint64_t src = s0; src < s1; ++src) {
        uint64_t cur = 0, at = 0;
        for (uint32_t r = 0; r < KT; ++r) {
          const uint32_t k = by_rank[r];
          const uint32_t q0 = tseg[src * (KT + 1) + k], L = tseg[src * (KT + 1) + k + 1] - q0;
          cur = dl_place(cur, L, sizeof(real), &at, packed);
          const uint32_t word = (uint32_t)((part[src] + at) / 4);
          dsegh[src * KT + r] = make_uint2(word, L);
          real *wp = reinterpret_cast<real *>(dlh.data() + word);
          uint16_t *op = reinterpret_cast<uint16_t *>(wp + L);
          for (uint32_t i = 0; i < L; ++i) {
            const uint32_t q = q0 + i, tgt = sm_syn[q] & 0xFFFFFFu, dly = sm_syn[q] >> 24;
            wp[i] = (real)sm_w[q];
            op[i] = (uint16_t)(dly * TS + (tgt - k * TS));
            dpos[q] = word + i * (uint32_t)(sizeof(real) / 4);
          }
        }
      }
    });
    uint32_t *pw = nullptr;
    uint2 *ps = nullptr;
    if (!dalloc(n, &pw, n->dl_words) || !dalloc(n, &ps, dsegh.size())) return hipErrorOutOfMemory;
    d.dlw = pw;
    d.dseg = ps;
    d.ts_magic = (uint32_t)((1ull << 32) / TS + 1);
    cp(pw, dlh.data(), dlh.size() * 4);
    cp(ps, dsegh.data(), dsegh.size() * sizeof(uint2));
    std::vector<uint32_t> tdp(n->S);
    parallel_ranges(n->S, nt, flat, [&](uint64_t lo, uint64_t hi, unsigned) {
      for (uint64_t q = lo; q < hi; ++q) tdp[q] = dpos[tm_perm[q]];
    });
    cp((void *)d.tm_dpos, tdp.data(), tdp.size() * 4);
    if (n->queues && e == hipSuccess) e = upload_queues(n, d, tseg, dsegh);
  }
  {
    // out-degree of every source per delay, for the event counts
    std::vector<uint32_t> od((size_t)n->NS * n->R, 0u);
    parallel_ranges(n->NS, nt, [&](uint64_t src) { return (uint64_t)sm_ptr[src]; },
                    [&](uint64_t s0, uint64_t s1, unsigned) {
                      for (uint64_t src = s0; src < s1; ++src)
                        for (uint32_t q = sm_ptr[src]; q < sm_ptr[src + 1]; ++q)
                          od[(size_t)src * n->R + (sm_syn[q] >> 24)]++;
                    });
    cp((void *)d.outdeg, od.data(), od.size() * 4);
  }
  cp((void *)d.tm_ptr, tm_ptr.data(), tm_ptr.size() * 4);
  cp((void *)d.tm_syn, tm_syn.data(), tm_syn.size() * 4);
  if (!n->blocked) {
    auto o = conv(tm_w);
    cp(d.tm_w, o.data(), o.size() * sizeof(real));
  } else {
    // blocks of the update: per tile, consecutive sources with at most
    // kApplySyn * 4 bytes of gradients into the tile (and at most kApplySrc
    // sources), tile-major; then where each target's run of a block's
    // sources starts in its row
    const uint32_t KT = d.KT, TS = d.TS;
    const uint64_t cap = (uint64_t)eprop::kApplySyn * 4 / sizeof(real);
    std::vector<uint32_t> ach, first(KT + 1, 0);
    for (uint32_t k = 0; k < KT; ++k) {
      first[k] = (uint32_t)(ach.size() / 3);
      uint32_t s0 = 0;
      uint64_t acc = 0;
      for (uint32_t src = 0; src < n->NS; ++src) {
        const uint32_t len = tseg[(size_t)src * (KT + 1) + k + 1] - tseg[(size_t)src * (KT + 1) + k];
        if (src > s0 && (acc + len > cap || src - s0 >= eprop::kApplySrc)) {
          if (acc) ach.insert(ach.end(), {k, s0, src});
          s0 = src;
          acc = 0;
        }
        acc += len;
      }
      if (acc) ach.insert(ach.end(), {k, s0, n->NS});
    }
    n->n_ach = (uint32_t)(ach.size() / 3);
    first[KT] = n->n_ach;
    // and each synapse's place in its block's source-major segments (the
    // segments of the block's sources into the tile, concatenated in source
    // order), so that the update reads 2 bytes instead of the synapse's
    // source and source-major position
    std::vector<uint32_t> trs((size_t)n->n_ach * TS, 0u);
    std::vector<uint16_t> loc(n->S, 0u);
    parallel_ranges(KT, nt, flat, [&](uint64_t k0, uint64_t k1, unsigned) {
      std::vector<uint32_t> cur(TS), pre, seg0;
      for (uint64_t k = k0; k < k1; ++k) {
        for (uint32_t t = 0; t < TS; ++t) {
          const uint64_t j = k * TS + t;
          cur[t] = j < n->J ? tm_ptr[j] : 0u;
        }
        for (uint32_t c = first[k]; c < first[k + 1]; ++c) {
          const uint32_t s0 = ach[3 * (size_t)c + 1], s1 = ach[3 * (size_t)c + 2];
          pre.assign(s1 - s0, 0u);
          seg0.assign(s1 - s0, 0u);
          uint32_t run = 0;
          for (uint32_t i = 0; i < s1 - s0; ++i) {
            const uint32_t *ts = tseg.data() + (size_t)(s0 + i) * (KT + 1) + k;
            pre[i] = run;
            seg0[i] = ts[0];
            run += ts[1] - ts[0];
          }
          for (uint32_t t = 0; t < TS; ++t) {
            const uint64_t j = k * TS + t;
            trs[(size_t)c * TS + t] = cur[t];
            if (j >= n->J) continue;
            for (; cur[t] < tm_ptr[j + 1]; ++cur[t]) {
              const uint32_t q = cur[t], src = tm_syn[q] & 0xFFFFFFu;
              if (src >= s1) break;
              loc[q] = (uint16_t)(pre[src - s0] + (tm_perm[q] - seg0[src - s0]));
            }
          }
        }
      }
    });
    uint32_t *pa = nullptr, *pt = nullptr;
    uint16_t *pl = nullptr;
    if (n->n_ach) {
      if (!dalloc(n, &pa, ach.size()) || !dalloc(n, &pt, trs.size()) || !dalloc(n, &pl, loc.size()))
        return hipErrorOutOfMemory;
      cp(pa, ach.data(), ach.size() * 4);
      cp(pt, trs.data(), trs.size() * 4);
      cp(pl, loc.data(), loc.size() * 2);
    }
    d.ach = pa;
    d.trs = pt;
    d.tm_loc = pl;
    if (e == hipSuccess) e = hipMemset(d.tsum, 0, (size_t)n->Jp * 8);
  }
  { auto o = conv(beta); cp((void *)d.beta_j, o.data(), o.size() * sizeof(real)); }
  d.any_alif = std::any_of(beta.begin(), beta.end(), [](double x) { return x != 0.0; }) ? 1 : 0;
  d.beta_a = (real)n->cfg.beta_a;
  const size_t KJ = (size_t)n->K * n->Jp;
  std::vector<double> wo(KJ, 0.0), fbp(KJ, 0.0);
  for (uint32_t k = 0; k < n->K; ++k)
    for (uint32_t j = 0; j < n->J; ++j) {
      wo[(size_t)k * n->Jp + j] = w_out[(size_t)k * n->J + j];
      fbp[(size_t)j * n->K + k] = fb[(size_t)j * n->K + k];
    }
  { auto o = conv(wo); cp(d.w_out, o.data(), o.size() * sizeof(real)); }
  { auto o = conv(fbp); cp(d.fb, o.data(), o.size() * sizeof(real)); }
  if (e == hipSuccess && n->S) e = hipMemset(d.gs, 0, n->S * sizeof(real));
  if (e == hipSuccess && n->S) e = hipMemset(d.gc, 0, n->S * sizeof(real));
  if (e == hipSuccess) e = hipMemset(d.gos, 0, KJ * sizeof(real));
  if (e == hipSuccess) e = hipMemset(d.goc, 0, KJ * sizeof(real));
  if (e == hipSuccess) e = hipMemset(d.cnt, 0, eprop::CNT_WORDS * 8);
  if (e == hipSuccess) {
    if (n->blocked) Launch<real>::input_bound_blocked(d, n->n_ach, nullptr);
    else Launch<real>::input_bound(d, nullptr);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (n->adam && e == hipSuccess) {
    // optimiser state: caller order -> target-major
    std::vector<double> m(n->S, 0.0), v(n->S, 0.0), mo(KJ, 0.0), vo(KJ, 0.0);
    if (opt) {
      // source-major for the blocked update, target-major otherwise (the
      // order in which the update kernel visits the synapses)
      const std::vector<uint32_t> &ord = n->blocked ? n->sm2caller : n->perm;
      for (uint64_t q = 0; q < n->S; ++q) {
        const uint32_t c = ord[q];
        const double *ms = c < n->S_in ? opt->m_in : opt->m_rec;
        const double *vs = c < n->S_in ? opt->v_in : opt->v_rec;
        const uint64_t o = c < n->S_in ? c : c - n->S_in;
        if (ms) m[q] = ms[o];
        if (vs) v[q] = vs[o];
      }
      for (uint32_t k = 0; k < n->K; ++k)
        for (uint32_t j = 0; j < n->J; ++j) {
          if (opt->m_out) mo[(size_t)k * n->Jp + j] = opt->m_out[(size_t)k * n->J + j];
          if (opt->v_out) vo[(size_t)k * n->Jp + j] = opt->v_out[(size_t)k * n->J + j];
        }
    }
    { auto o = conv(m); cp(d.adam_m, o.data(), o.size() * sizeof(real)); }
    { auto o = conv(v); cp(d.adam_v, o.data(), o.size() * sizeof(real)); }
    { auto o = conv(mo); cp(d.adam_mo, o.data(), o.size() * sizeof(real)); }
    { auto o = conv(vo); cp(d.adam_vo, o.data(), o.size() * sizeof(real)); }
  }
  return e;
}

}  // namespace

extern "C" {

const char *eprop_status_string(int32_t s) {
  switch (s) {
    case EPROP_OK: return "ok";
    case EPROP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case EPROP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case EPROP_ERR_DEVICE: return "device error";
    case EPROP_ERR_STATE: return "call not valid in the handle's state";
    case EPROP_ERR_CAPACITY: return "batch exceeds the configured capacity";
    case EPROP_ERR_NUMERIC: return "non-finite loss";
    case EPROP_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *eprop_last_error(const eprop_network *net) {
  return net ? net->err.c_str() : g_create_error.c_str();
}

void eprop_destroy_network(eprop_network *net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->stream);
  for (auto &g : net->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto &e : net->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : net->tev)
    if (e) (void)hipEventDestroy(e);
  if (net->cap_stream) (void)hipStreamDestroy(net->cap_stream);
  for (void *p : net->allocs) dfree(net, p);
  delete net;
}

// The body of eprop_create_network; *partial is the handle under
// construction, for the caller to release if a host allocation throws.
static eprop_status create_network(const eprop_config *cfg, const eprop_projection *in_rec,
                                   const eprop_projection *rec_rec, const double *w_out,
                                   const double *feedback, const eprop_optimizer_state *opt,
                                   void *hip_stream, eprop_network **out_net, eprop_network **partial) {
  std::string msg;
  eprop_status st = check_config(cfg, msg);
  if (st == EPROP_OK) st = check_projection(in_rec, cfg->n_in, cfg->n_rec, cfg->max_delay, false, "in_rec", msg);
  if (st == EPROP_OK) st = check_projection(rec_rec, cfg->n_rec, cfg->n_rec, cfg->max_delay, true, "rec_rec", msg);
  if (st == EPROP_OK && (in_rec->nnz + rec_rec->nnz) >= (1ull << 32)) {
    msg = "2^32 or more synapses";
    st = EPROP_ERR_INVALID_ARGUMENT;
  }
  if (st == EPROP_OK && (!w_out || !feedback)) {
    msg = "NULL w_out or feedback";
    st = EPROP_ERR_INVALID_ARGUMENT;
  }
  if (st == EPROP_OK) {
    for (size_t i = 0; i < (size_t)cfg->n_out * cfg->n_rec; ++i)
      if (!is_finite(w_out[i]) || !is_finite(feedback[i])) {
        msg = "non-finite w_out or feedback";
        st = EPROP_ERR_INVALID_ARGUMENT;
        break;
      }
  }
  if (st != EPROP_OK) {
    g_create_error = msg;
    return st;
  }

  // graph in both orders (pure host work); duplicates found on the way
  const uint32_t I = cfg->n_in, J = cfg->n_rec, NS = I + J;
  const uint64_t S_in = in_rec->nnz, S_rec = rec_rec->nnz, S = S_in + S_rec;
  std::vector<uint32_t> sm_ptr(NS + 1), sm_syn(S), tm_ptr(J + 1, 0), tm_syn(S), tm_perm(S);
  std::vector<double> sm_w(S), tm_w(S);
  for (uint32_t i = 0; i <= I; ++i) sm_ptr[i] = (uint32_t)in_rec->row_ptr[i];
  for (uint32_t i = 1; i <= J; ++i) sm_ptr[I + i] = (uint32_t)(S_in + rec_rec->row_ptr[i]);
  // internal source-major order: each row sorted by target (stable), so that
  // the targets of one tile form one contiguous segment of the row.  Threads
  // take consecutive ranges of sources of about equal synapse counts and
  // count the targets of their range; the target-major order (rows sorted
  // by source) is then filled by the same ranges into disjoint slots.
  std::vector<uint32_t> sm2caller(S);
  const unsigned nt = S >= (1u << 22) ? host_threads() : 1u;
  std::vector<std::vector<uint32_t>> tcount(nt);
  auto sm_weight = [&](uint64_t src) { return (uint64_t)sm_ptr[src]; };
  parallel_ranges(NS, nt, sm_weight, [&](uint64_t s0, uint64_t s1, unsigned t) {
    std::vector<uint32_t> &cnt = tcount[t];
    cnt.assign(J, 0u);
    std::vector<uint32_t> idx;
    for (uint64_t src = s0; src < s1; ++src) {
      const bool in = src < I;
      const eprop_projection *p = in ? in_rec : rec_rec;
      const uint64_t lo = in ? in_rec->row_ptr[src] : rec_rec->row_ptr[src - I];
      const uint64_t hi = in ? in_rec->row_ptr[src + 1] : rec_rec->row_ptr[src - I + 1];
      idx.resize(hi - lo);
      for (uint64_t q = lo; q < hi; ++q) idx[q - lo] = (uint32_t)q;
      bool sorted = true;
      for (size_t i = 1; i < idx.size() && sorted; ++i) sorted = p->col[idx[i - 1]] <= p->col[idx[i]];
      if (!sorted)
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return p->col[x] < p->col[y]; });
      const uint64_t base = in ? 0 : S_in;
      for (size_t i = 0; i < idx.size(); ++i) {
        const uint64_t pos = sm_ptr[src] + i, q = idx[i];
        const uint32_t d = p->delay ? p->delay[q] : 1u;
        sm_syn[pos] = p->col[q] | (d << 24);
        sm_w[pos] = p->w[q];
        sm2caller[pos] = (uint32_t)(base + q);
        cnt[p->col[q]]++;
      }
    }
  });
  // slot of range t within target j's row: after the counts of ranges < t
  for (uint32_t j = 0; j < J; ++j) {
    uint32_t run = 0;
    for (unsigned t = 0; t < nt; ++t) {
      const uint32_t c = tcount[t][j];
      tcount[t][j] = run;
      run += c;
    }
    tm_ptr[j + 1] = tm_ptr[j] + run;
  }
  std::atomic<bool> dup{false};
  parallel_ranges(NS, nt, sm_weight, [&](uint64_t s0, uint64_t s1, unsigned t) {
    std::vector<uint32_t> &fill = tcount[t];
    const std::vector<uint32_t> start(fill);
    for (uint64_t src = s0; src < s1 && !dup.load(std::memory_order_relaxed); ++src)
      for (uint32_t q = sm_ptr[src]; q < sm_ptr[src + 1]; ++q) {
        const uint32_t tgt = sm_syn[q] & 0xFFFFFFu;
        const uint32_t pos = tm_ptr[tgt] + fill[tgt]++;
        // a repeated pair lands in consecutive slots of this range's part of the row
        if (pos > tm_ptr[tgt] + start[tgt] && (tm_syn[pos - 1] & 0xFFFFFFu) == src) {
          dup.store(true);
          break;
        }
        tm_syn[pos] = (uint32_t)src | (sm_syn[q] & 0xFF000000u);
        tm_w[pos] = sm_w[q];
        tm_perm[pos] = q;
      }
  });
  tcount.clear();
  tcount.shrink_to_fit();
  if (dup) {
    g_create_error = "duplicate synapse between one pair of neurons";
    return EPROP_ERR_INVALID_ARGUMENT;
  }

  // device
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    g_create_error = "no HIP device";
    return EPROP_ERR_DEVICE;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    g_create_error = "cannot query the HIP device";
    return EPROP_ERR_DEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("library built for gfx950, device is ") + prop.gcnArchName;
    return EPROP_ERR_DEVICE;
  }

  eprop_network *n = new (std::nothrow) eprop_network();
  if (!n) { g_create_error = "host allocation failed"; return EPROP_ERR_OUT_OF_MEMORY; }
  *partial = n;
  n->cfg = *cfg;
  n->cfg.is_alif = nullptr;
  n->I = I; n->J = J; n->K = cfg->n_out; n->NS = NS;
  n->Jw = (J + 63) / 64; n->Jp = n->Jw * 64; n->Iw = std::max<uint32_t>(1, (I + 63) / 64);
  n->R = cfg->max_delay + 1; n->Tcap = cfg->max_steps; n->Tp = round_up(n->Tcap + 1, 16);
  n->Bcap = cfg->max_trials;
  n->S_in = S_in; n->S_rec = S_rec; n->S = S;
  n->fp64 = cfg->precision == EPROP_FP64;
  n->gather = cfg->delivery == EPROP_DELIVERY_GATHER || (cfg->delivery == EPROP_DELIVERY_AUTO && n->fp64);
  n->adam = cfg->optimizer == EPROP_OPT_ADAM;
  n->use_graph = (cfg->flags & EPROP_FLAG_NO_GRAPH) == 0;
  n->n_ref = (uint32_t)std::lround(cfg->t_ref / cfg->dt);
  // exact-integration propagators (eq. lif_update, eq. spike-threshold-adaptation,
  // eq. leaky_integrator)
  n->alpha = std::exp(-cfg->dt / cfg->tau_m);
  n->rho = std::exp(-cfg->dt / cfg->tau_a);
  n->kappa = std::exp(-cfg->dt / cfg->tau_out);
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->perm = tm_perm;
  n->adam_step = opt ? opt->step : 0;
  n->h_in_ptr.reserve(n->Bcap + 1);
  n->h_f_ptr.reserve(n->Bcap + 1);
  n->h_loss.reserve(n->Bcap);
  n->h_pred.reserve(n->Bcap);
  n->last_T.reserve(n->Bcap);
  n->shapes.block = 256;
  n->shapes.fwd_variant = 0;
  n->shapes.adj_block = cfg->n_out > 16 ? 64 : 256;
  n->shapes.syn_var = 0;
  n->autotune_pending = (cfg->flags & EPROP_AUTOTUNE) != 0;
  {
    // synapse kernel: a block per (target, chunk of trials); the chunk's
    // archive rows (Ts entries each, plus a zero tail of R) should fit 16 KB
    // of LDS and must fit 64 KB; small networks with many trials use smaller
    // chunks to fill the device
    const size_t rs = n->fp64 ? 8 : 4;
    n->Ts = round_up(n->Tcap + n->R, 4);
    const size_t row = (size_t)n->Ts * rs;
    if (row + (size_t)n->R * rs > 65536) {
      g_create_error = "trials longer than the synapse kernel's LDS rows allow (max_steps too large)";
      delete n;
      return EPROP_ERR_UNSUPPORTED;
    }
    uint32_t g = (uint32_t)std::max<size_t>(1, (16384 - std::min<size_t>(16384, (size_t)n->R * rs)) / row);
    g = std::min<uint32_t>(std::min<uint32_t>(g, n->Bcap), 8);
    const uint64_t par = (uint64_t)n->Bcap * J / 4096;
    g = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, par));
    n->shapes.ginst = g;
    const double indeg = (double)S / J;
    uint32_t sb = 64;
    while (sb < 256 && sb < indeg) sb += 64;
    n->shapes.syn_block = sb;
  }
  n->sm2caller = std::move(sm2caller);
  parallel_ranges(S, nt, [](uint64_t q) { return q; }, [&](uint64_t lo, uint64_t hi, unsigned) {
    for (uint64_t q = lo; q < hi; ++q) n->perm[q] = n->sm2caller[tm_perm[q]];
  });
  // Tiles of the persistent forward kernel: as many neurons per workgroup as
  // LDS allows, but enough tiles to spread the trials over the device; small
  // networks keep a whole trial in one workgroup (no inter-workgroup barrier).
  uint32_t TS = n->Jp, KT = 1, tile_block = 64, ring_bytes = 8, ptab_cap = 4096;
  if (!n->gather) {
    size_t lds = prop.sharedMemPerBlock;
    if (prop.sharedMemPerBlockOptin > lds) lds = prop.sharedMemPerBlockOptin;
    if (prop.maxSharedMemoryPerMultiProcessor > 0 && lds > prop.maxSharedMemoryPerMultiProcessor)
      lds = prop.maxSharedMemoryPerMultiProcessor;
    const size_t fixed = 1024 + 4 * 1025;  // static LDS of the kernel (tile count prefix) and slack
    // the tile size is chosen with a piece table of 3072 entries (24 KB: at
    // least 3 per thread), which grows to 4096 where LDS has room
    auto smem_of = [&](uint32_t ts, uint32_t rb, uint32_t cap = 3072) {
      return n->fp64 ? Launch<double>::tile_smem(ts, n->R, rb, cap) : Launch<float>::tile_smem(ts, n->R, rb, cap);
    };
    auto ts_max = [&](uint32_t rb) {  // largest tile (multiple of 64) that fits LDS
      uint32_t ts = 64;
      while (smem_of(ts + 64, rb) + fixed <= lds) ts += 64;
      return smem_of(ts, rb) + fixed <= lds ? ts : 0u;
    };
    const uint32_t cu = std::max(1, prop.multiProcessorCount);
    const uint32_t want = std::max<uint32_t>(1, cu / n->Bcap);
    uint32_t ts_par = round_up((J + want - 1) / want, 64);
    ts_par = std::max<uint32_t>(ts_par, std::min<uint32_t>(n->Jp, 512));
    ts_par = std::min(ts_par, n->Jp);
    // FP32: 32-bit fixed-point ring entries (each arrival rounded to half a
    // quantum, 2^-31 of the input bound: finer than an FP32 running sum of
    // the same arrivals, whose additions round at 2^-24 of it); FP64: double
    ring_bytes = n->fp64 ? 8u : 4u;
    const uint32_t ts_lds = ts_max(ring_bytes);
    if (ts_lds < 64) {
      g_create_error = "not enough LDS for a tile of 64 neurons";
      delete n;
      return EPROP_ERR_UNSUPPORTED;
    }
    TS = std::max<uint32_t>(std::min(ts_lds, ts_par), 64);
    KT = (n->Jp + TS - 1) / TS;
    tile_block = std::min<uint32_t>(1024, TS);
    if (KT > tile_block) {  // every tile's count is read by one thread of each tile
      g_create_error = "too many tiles per trial for the tiled forward kernel";
      delete n;
      return EPROP_ERR_UNSUPPORTED;
    }
    ptab_cap = smem_of(TS, ring_bytes, 4096) + fixed <= lds ? 4096u : 3072u;
    // ring offsets d * TS + (target - k * TS) in 16 bits; segment lengths
    // within the piece entries' 26-bit field
    uint64_t max_row = 0;
    for (uint32_t src = 0; src < NS; ++src) max_row = std::max<uint64_t>(max_row, sm_ptr[src + 1] - sm_ptr[src]);
    if ((uint64_t)n->R * TS > 65536 || max_row * (n->fp64 ? 4 : 2) >= (1ull << 26)) {
      g_create_error = "delays or rows too long for the delivery table";
      delete n;
      return EPROP_ERR_UNSUPPORTED;
    }
    n->tile_smem = smem_of(TS, ring_bytes, ptab_cap);
    // blocked transposition for the update where source rows are dense within
    // a tile (at least 4 synapses per source and tile on average)
    const size_t blk_lds = n->fp64 ? Launch<double>::apply_blocked_smem(TS) : Launch<float>::apply_blocked_smem(TS);
    n->blocked = TS <= eprop::kApplyMaxTile && blk_lds <= lds &&
                 (double)S >= 4.0 * (double)NS * (double)((n->Jp + TS - 1) / TS);
  }
  n->shapes.tile_block = tile_block;
  n->n32.TS = n->n64.TS = TS;
  n->n32.KT = n->n64.KT = KT;
  n->n32.ring_bytes = n->n64.ring_bytes = ring_bytes;
  n->n32.ptab_cap = n->n64.ptab_cap = ptab_cap;
  n->blk = std::min<uint32_t>(n->gather ? 50 : 250, n->Tcap);

  std::vector<double> beta(n->Jp, 0.0);
  for (uint32_t j = 0; j < J; ++j) beta[j] = (cfg->is_alif && cfg->is_alif[j]) ? cfg->beta_a : 0.0;

  {
    // The per-trial archives hold whole trials (the gradient of a trial is
    // formed once it is complete), so they grow as max_trials x max_steps x
    // neurons: psi and phi, spike bitsets (recurrent, forced, input),
    // spike-time lists, the per-source spike table and the readout rows.
    const size_t rs = n->fp64 ? 8 : 4, B = n->Bcap, T1 = (size_t)n->Tcap + 1, Lc = round_up(n->Tcap, 8);
    const size_t per_trial = T1 * n->Jp * rs + (size_t)n->Jp * n->Tp * rs + 2 * T1 * n->Jw * 8 +
                             (size_t)n->Tcap * n->Iw * 8 + 2 * (size_t)n->NS * Lc * 2 + 5 * (T1 + 1) * n->K * 8;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && B * per_trial > free_b) {
      g_create_error = "the trial archives need " + std::to_string(B * per_trial >> 20) + " MiB (" +
                       std::to_string(per_trial >> 20) + " MiB per trial of max_steps steps) and the device has " +
                       std::to_string(free_b >> 20) + " MiB free: lower max_trials or max_steps";
      delete n;
      return EPROP_ERR_CAPACITY;
    }
  }
  {
    // per-tile queues (FP32 scatter delivery): built where recurrent rows are
    // sparse across tiles (fewer than 4 synapses per source and tile on
    // average) and they fit a quarter of the free memory, or when asked for
    const bool want = (cfg->flags & EPROP_SCATTER_QUEUES) != 0;
    const bool able = !n->gather && !n->fp64 && KT > 1 && n->S > 0 && n->S < (1ull << 32);
    if (want && !able) {
      g_create_error = "EPROP_SCATTER_QUEUES needs FP32 scatter delivery, more than one tile per trial and "
                       "fewer than 2^32 synapses";
      delete n;
      return EPROP_ERR_UNSUPPORTED;
    }
    const bool sparse = (double)n->S_rec < 4.0 * (double)J * (double)KT;
    if (able && !(cfg->flags & EPROP_SCATTER_LOOKUP) && (want || sparse)) {
      const size_t kt2 = (size_t)KT * KT;
      const size_t bytes = (size_t)n->Bcap * 2 * n->S * 8 + (n->S_rec + (size_t)I * KT) * 8 + ((size_t)J + 1) * 4 +
                           2 * kt2 * 4 + (size_t)n->Bcap * 2 * kt2 * 8;
      size_t free_b = 0, total_b = 0;
      const bool known = hipMemGetInfo(&free_b, &total_b) == hipSuccess;
      if (want && known && bytes > free_b) {
        g_create_error = "the per-tile queues need " + std::to_string(bytes >> 20) + " MiB and the device has " +
                         std::to_string(free_b >> 20) + " MiB free";
        delete n;
        return EPROP_ERR_CAPACITY;
      }
      n->queues = want || (known && bytes <= free_b / 4);
    }
    if (n->queues) n->shapes.fwd_variant = eprop::kQueueVariant;
  }
  bool ok = n->fp64 ? alloc_state(n, n->n64) : alloc_state(n, n->n32);
  ok = ok && dalloc(n, &n->d_T, n->Bcap) && dalloc(n, &n->d_label, n->Bcap) && dalloc(n, &n->d_in_ptr, n->Bcap + 1) &&
       dalloc(n, &n->d_forced_ptr, n->Bcap + 1);
  if (!ok) {
    g_create_error = "out of device memory";
    eprop_destroy_network(n);
    return EPROP_ERR_OUT_OF_MEMORY;
  }
  // tile segments of every source row
  std::vector<uint32_t> tseg;
  if (!n->gather) {
    tseg.resize((size_t)NS * (KT + 1));
    parallel_ranges(NS, nt, sm_weight, [&](uint64_t s0, uint64_t s1, unsigned) {
      for (uint64_t src = s0; src < s1; ++src) {
        uint32_t q = sm_ptr[src];
        const uint32_t hi = sm_ptr[src + 1];
        for (uint32_t k = 0; k <= KT; ++k) {
          const uint64_t lo_t = (uint64_t)k * TS;
          while (q < hi && (sm_syn[q] & 0xFFFFFFu) < lo_t) ++q;
          tseg[(size_t)src * (KT + 1) + k] = q;
        }
        tseg[(size_t)src * (KT + 1) + KT] = hi;
      }
    });
  }
  hipError_t e = hipSuccess;
  if (!n->gather) {
    const uint32_t rb = n->n32.ring_bytes ? n->n32.ring_bytes : n->n64.ring_bytes;
    e = n->fp64 ? Launch<double>::allow_smem(n->tile_smem, rb) : Launch<float>::allow_smem(n->tile_smem, rb);
    int per_cu = 0;
    if (e == hipSuccess)
      e = n->fp64 ? Launch<double>::resident(tile_block, n->tile_smem, rb, &per_cu)
                  : Launch<float>::resident(tile_block, n->tile_smem, rb, &per_cu);
    if (e == hipSuccess && (uint64_t)per_cu * prop.multiProcessorCount < KT) {
      g_create_error = "the tiles of one trial cannot be resident together on this device";
      eprop_destroy_network(n);
      return EPROP_ERR_UNSUPPORTED;
    }
    // trials per forward launch: as many as are resident together
    const uint64_t resident_trials = (uint64_t)per_cu * prop.multiProcessorCount / KT;
    n->shapes.fwd_trials = (uint32_t)std::min<uint64_t>(n->Bcap, std::max<uint64_t>(1, resident_trials));
  }
  if (e == hipSuccess)
    e = n->fp64 ? upload(n, n->n64, sm_ptr, tseg, sm_syn, sm_w, tm_ptr, tm_syn, tm_perm, tm_w, beta, w_out,
                         feedback, opt)
                : upload(n, n->n32, sm_ptr, tseg, sm_syn, sm_w, tm_ptr, tm_syn, tm_perm, tm_w, beta, w_out,
                         feedback, opt);
  if (e == hipErrorNotSupported && !g_create_error.empty()) {  // a size the tables cannot address
    eprop_destroy_network(n);
    return EPROP_ERR_UNSUPPORTED;
  }
  if (e == hipSuccess) {  // this device's staging array of the no-allocation batch call (device current)
    n->scratch = static_cast<uint8_t *>(eprop::scratch_address(dev, &e));
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&n->cap_stream, hipStreamNonBlocking);
  for (auto &ev : n->ev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  for (auto &ev : n->tev)
    if (e == hipSuccess) e = hipEventCreate(&ev);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    g_create_error = std::string("device error during setup: ") + hip_msg(e);
    eprop_destroy_network(n);
    return EPROP_ERR_DEVICE;
  }
  *partial = nullptr;
  *out_net = n;
  return EPROP_OK;
}

eprop_status eprop_create_network(const eprop_config *cfg, const eprop_projection *in_rec,
                                  const eprop_projection *rec_rec, const double *w_out,
                                  const double *feedback, const eprop_optimizer_state *opt,
                                  void *hip_stream, eprop_network **out_net) {
  g_create_error.clear();
  if (!out_net) { g_create_error = "NULL out_net"; return EPROP_ERR_INVALID_ARGUMENT; }
  *out_net = nullptr;
  eprop_network *partial = nullptr;
  try {
    return create_network(cfg, in_rec, rec_rec, w_out, feedback, opt, hip_stream, out_net, &partial);
  } catch (const std::exception &x) {
    g_create_error = host_failure(x);
  } catch (...) {
    g_create_error = "host failure";
  }
  if (partial) eprop_destroy_network(partial);
  return EPROP_ERR_OUT_OF_MEMORY;
}

}  // extern "C"

namespace {

// Validates a batch on the host.  Device-memory arrays are checked by the
// staging kernels; their in_ptr / forced_ptr are copied and checked here.
eprop_status check_batch(eprop_network *n, const eprop_batch *b, std::vector<uint64_t> &in_ptr,
                         std::vector<uint64_t> &f_ptr, uint32_t &t_max, std::string &msg) {
  auto bad = [&](const char *m) { msg = m; return EPROP_ERR_INVALID_ARGUMENT; };
  if (b->n_trials < 1) return bad("n_trials must be >= 1");
  if (b->n_trials > n->Bcap) { msg = "n_trials exceeds max_trials"; return EPROP_ERR_CAPACITY; }
  if (b->memory != EPROP_MEM_HOST && b->memory != EPROP_MEM_DEVICE) return bad("unknown memory kind");
  if (b->flags & ~(uint32_t)(EPROP_BATCH_TRAIN | EPROP_BATCH_PROFILE | EPROP_RECORD_SPIKES | EPROP_RECORD_TRACES |
                             EPROP_BATCH_TIME_DRIVEN))
    return bad("unknown batch flag");
  if (!b->n_steps) return bad("NULL n_steps");
  t_max = 0;
  for (uint32_t i = 0; i < b->n_trials; ++i) {
    if (b->n_steps[i] < 1) return bad("trial with 0 steps");
    if (b->n_steps[i] > n->Tcap) { msg = "trial longer than max_steps"; return EPROP_ERR_CAPACITY; }
    t_max = std::max(t_max, b->n_steps[i]);
  }
  if (b->step_stride < t_max) return bad("step_stride smaller than the longest trial");
  if (n->cfg.loss == EPROP_LOSS_MSE && !b->target) return bad("MSE needs a target");
  if (n->cfg.loss == EPROP_LOSS_SOFTMAX_CE || n->cfg.loss == EPROP_LOSS_TEMPORAL_MSE) {
    if (!b->label) return bad("classification losses need labels");
    for (uint32_t i = 0; i < b->n_trials; ++i)
      if (b->label[i] >= n->K) return bad("label out of range");
  }
  if (!b->in_ptr) return bad("NULL in_ptr");
  if (b->n_in_spikes > 0 && (!b->in_step || !b->in_src)) return bad("NULL in_step or in_src");
  if (b->n_in_spikes >= (1ull << 40)) return bad("too many input spikes");
  const bool dev = b->memory == EPROP_MEM_DEVICE;
  in_ptr.assign(b->n_trials + 1, 0);
  if (dev) {
    if (hipMemcpy(in_ptr.data(), b->in_ptr, in_ptr.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      return bad("in_ptr is not readable device memory");
    }
  } else {
    std::memcpy(in_ptr.data(), b->in_ptr, in_ptr.size() * 8);
  }
  if (in_ptr[0] != 0 || in_ptr[b->n_trials] != b->n_in_spikes) return bad("in_ptr must span 0..n_in_spikes");
  for (uint32_t i = 0; i < b->n_trials; ++i)
    if (in_ptr[i] > in_ptr[i + 1]) return bad("in_ptr decreases");
  if (!dev) {
    for (uint32_t i = 0; i < b->n_trials; ++i)
      for (uint64_t e = in_ptr[i]; e < in_ptr[i + 1]; ++e) {
        if (b->in_step[e] >= b->n_steps[i] || b->in_src[e] >= n->I) return bad("input spike out of range");
        if (e > in_ptr[i]) {
          const uint32_t ps = b->in_step[e - 1], pi = b->in_src[e - 1];
          if (!(ps < b->in_step[e] || (ps == b->in_step[e] && pi < b->in_src[e])))
            return bad("input spikes not strictly sorted by (step, source)");
        }
      }
  }
  f_ptr.clear();
  if (b->forced_ptr) {
    if (b->n_forced > 0 && (!b->forced_step || !b->forced_neuron)) return bad("NULL forced arrays");
    f_ptr.assign(b->n_trials + 1, 0);
    if (dev) {
      if (hipMemcpy(f_ptr.data(), b->forced_ptr, f_ptr.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return bad("forced_ptr is not readable device memory");
      }
    } else {
      std::memcpy(f_ptr.data(), b->forced_ptr, f_ptr.size() * 8);
    }
    if (f_ptr[0] != 0 || f_ptr[b->n_trials] != b->n_forced) return bad("forced_ptr must span 0..n_forced");
    for (uint32_t i = 0; i < b->n_trials; ++i) {
      if (f_ptr[i] > f_ptr[i + 1]) return bad("forced_ptr decreases");
      if (!dev)
        for (uint64_t e = f_ptr[i]; e < f_ptr[i + 1]; ++e)
          if (b->forced_step[e] < 1 || b->forced_step[e] > b->n_steps[i] || b->forced_neuron[e] >= n->J)
            return bad("forced spike out of range");
    }
  }
  return EPROP_OK;
}

template <typename real>
void record_block(eprop_network *n, DevNet<real> &d, bool forced, hipStream_t s) {
  if (n->gather) {
    for (uint32_t o = 1; o <= n->blk; ++o) Launch<real>::neuron_gather(d, o, forced, s);
  } else {
    Launch<real>::forward_tiled(d, n->blk, forced, n->shapes, n->tile_smem, s);
  }
  eprop::launch_advance(d.ctl, n->blk, s);
}

template <typename real>
hipError_t ensure_graph(eprop_network *n, DevNet<real> &d, bool forced) {
  hipGraphExec_t &ge = n->gexec[forced ? 1 : 0];
  if (ge) return hipSuccess;
  hipError_t e = hipStreamBeginCapture(n->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  record_block(n, d, forced, n->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(n->cap_stream, &g);
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

void drop_graphs(eprop_network *n) {
  for (auto &g : n->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Returns a buffer from dalloc before the handle is destroyed.
void release(eprop_network *n, void *p) {
  auto it = std::find(n->allocs.begin(), n->allocs.end(), p);
  if (it != n->allocs.end()) n->allocs.erase(it);
  dfree(n, p);
}

// The samples of an online batch joined into one run (host arrays).
struct OnlineCtx {
  uint32_t n_samples = 0;
  std::vector<uint32_t> off, label;   // off[c]: steps before sample c
};

template <typename real>
eprop_status run_online(eprop_network *n, DevNet<real> &d, const eprop_batch *b, eprop_batch_result *res,
                        const OnlineCtx &oc, bool forced, bool prof, hipError_t &e);

// noalloc: eprop_simulate_batch_noalloc (host-memory batch arrays staged in
// the device's static array, no device allocation, no graph instantiation,
// no autotuning in this call).
template <typename real>
eprop_status simulate(eprop_network *n, DevNet<real> &d, const eprop_batch *b, eprop_batch_result *res,
                      const OnlineCtx *oc = nullptr, bool noalloc = false) {
  std::string msg;
  std::vector<uint64_t> &in_ptr = n->h_in_ptr, &f_ptr = n->h_f_ptr;
  uint32_t t_max = 0;
  eprop_status st = check_batch(n, b, in_ptr, f_ptr, t_max, msg);
  if (st != EPROP_OK) {
    set_fail(n, msg);
    return st;
  }
  const uint32_t ntr = b->n_trials;
  const bool dev = b->memory == EPROP_MEM_DEVICE;
  const bool forced = b->forced_ptr != nullptr;
  const bool train = (b->flags & EPROP_BATCH_TRAIN) != 0;
  const bool prof = (b->flags & EPROP_BATCH_PROFILE) != 0;
  const bool time_driven = train && (b->flags & EPROP_BATCH_TIME_DRIVEN) != 0;
  if (time_driven && n->cfg.reg_mode == EPROP_REG_MOVING_AVERAGE && n->cfg.c_reg != 0.0) {
    set_fail(n, "the time-driven baseline has no moving-average regulariser");
    return EPROP_ERR_UNSUPPORTED;
  }
  if (time_driven) {
    const size_t need = (size_t)n->Bcap * n->Jp * n->Tp * sizeof(real);  // neuron-major [b][j][Tp]
    uint8_t *lb = static_cast<uint8_t *>(n->Lbuf);
    if (!dgrow(n, &lb, &n->cap_Lbuf, need)) {
      set_fail(n, "out of device memory for the time-driven learning signal");
      return EPROP_ERR_OUT_OF_MEMORY;
    }
    n->Lbuf = lb;
  }
  hipStream_t s = n->stream;
  hipError_t e = hipSuccess;
  auto H2D = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  auto MS = [&](void *dst, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemsetAsync(dst, 0, bytes, s);
  };

  // batch arrays: library copies for host memory, caller's for device memory
  uint32_t *st_in_step = n->d_in_step, *st_in_src = n->d_in_src, *st_f_step = n->d_forced_step,
           *st_f_neuron = n->d_forced_neuron;
  double *st_target = n->d_target;
  uint8_t *st_window = n->d_window;
  if (!dev && noalloc) {
    // consecutive 256-byte aligned pieces of the static staging array
    const size_t nt = (size_t)ntr * b->step_stride;
    const size_t sizes[6] = {b->n_in_spikes * 4, b->n_in_spikes * 4, b->target ? nt * n->K * 8 : 0,
                             b->window ? nt : 0, forced ? b->n_forced * 4 : 0, forced ? b->n_forced * 4 : 0};
    size_t off[6], used = 0;
    for (int i = 0; i < 6; ++i) {
      off[i] = used;
      used += (sizes[i] + 255) / 256 * 256;
    }
    if (used > eprop::kScratchBytes) {
      set_fail(n, "the batch's host arrays (" + std::to_string(used) + " bytes staged) exceed the " +
                      std::to_string(eprop::kScratchBytes) + "-byte staging array of eprop_simulate_batch_noalloc");
      return EPROP_ERR_CAPACITY;
    }
    st_in_step = reinterpret_cast<uint32_t *>(n->scratch + off[0]);
    st_in_src = reinterpret_cast<uint32_t *>(n->scratch + off[1]);
    st_target = reinterpret_cast<double *>(n->scratch + off[2]);
    st_window = n->scratch + off[3];
    st_f_step = reinterpret_cast<uint32_t *>(n->scratch + off[4]);
    st_f_neuron = reinterpret_cast<uint32_t *>(n->scratch + off[5]);
  } else if (!dev) {
    const size_t nt = (size_t)ntr * b->step_stride;
    bool ok = dgrow(n, &n->d_in_step, &n->cap_in_step, b->n_in_spikes) &&
              dgrow(n, &n->d_in_src, &n->cap_in_src, b->n_in_spikes);
    if (ok && b->target) ok = dgrow(n, &n->d_target, &n->cap_target, nt * n->K);
    if (ok && b->window) ok = dgrow(n, &n->d_window, &n->cap_window, nt);
    if (ok && forced)
      ok = dgrow(n, &n->d_forced_step, &n->cap_f_step, b->n_forced) &&
           dgrow(n, &n->d_forced_neuron, &n->cap_f_neuron, b->n_forced);
    if (!ok) {
      set_fail(n, "out of device memory for the batch");
      return EPROP_ERR_OUT_OF_MEMORY;
    }
    st_in_step = n->d_in_step;
    st_in_src = n->d_in_src;
    st_target = n->d_target;
    st_window = n->d_window;
    st_f_step = n->d_forced_step;
    st_f_neuron = n->d_forced_neuron;
  }
  d.T = n->d_T;
  d.label = n->d_label;
  d.step_stride = b->step_stride;
  if (dev) {
    d.in_ptr = b->in_ptr;
    d.in_step = b->in_step;
    d.in_src = b->in_src;
    d.target = b->target;
    d.window = b->window;
    d.forced_ptr = b->forced_ptr;
    d.forced_step = b->forced_step;
    d.forced_neuron = b->forced_neuron;
  } else {
    d.in_ptr = n->d_in_ptr;
    d.in_step = st_in_step;
    d.in_src = st_in_src;
    d.target = b->target ? st_target : nullptr;
    d.window = b->window ? st_window : nullptr;
    d.forced_ptr = n->d_forced_ptr;
    d.forced_step = st_f_step;
    d.forced_neuron = st_f_neuron;
  }

  struct {
    uint32_t w[eprop::CTL_WORDS];
    const uint32_t *in_src;
  } ctl{};
  ctl.w[eprop::CTL_T0] = 0;
  ctl.w[eprop::CTL_NTRIALS] = ntr;
  ctl.w[eprop::CTL_ERR] = 0;
  ctl.in_src = d.in_src;
  const size_t T1 = (size_t)n->Tcap + 1;
  // per-batch state from zero (trials start from rest) and staged inputs;
  // run again by the autotuner before each timed forward pass
  auto restage = [&]() {
    if (n->queues) {  // the pass's queue tags CTL_TAG0 + t, none used since the queues were last cleared
      if ((uint64_t)n->q_since + t_max + 1 > 65535) {
        MS(d.q_ev, (size_t)n->Bcap * 2 * d.q_len * 8);
        MS(d.q_hdr, (size_t)n->Bcap * 2 * d.KT * d.KT * 8);
        n->q_since = 0;
      }
      ctl.w[eprop::CTL_TAG0] = n->q_since;
      n->q_since += t_max;
    }
    H2D(d.ctl, &ctl, sizeof(ctl));
    MS(d.v, (size_t)ntr * n->Jp * sizeof(real));
    MS(d.a, (size_t)ntr * n->Jp * sizeof(real));
    MS(d.nst, (size_t)ntr * n->Jp);
    MS(d.ring, (size_t)ntr * n->R * n->Jp * d.ring_bytes);
    MS(d.in_bits, (size_t)ntr * n->Tcap * n->Iw * 8);
    MS(d.spk_cnt, (size_t)ntr * n->NS * 4);
    if (!n->gather) {  // tags of an earlier batch must not match
      MS(d.pub_list, (size_t)ntr * 2 * n->Jp * 8);
      MS(d.pub_cnt, (size_t)ntr * 2 * d.KT * 8);
    }
    MS(d.cnt, eprop::CNT_WORDS * 8);
    MS(d.evcnt, 64 * 8);
    if (forced) MS(d.forced_bits, (size_t)ntr * T1 * n->Jw * 8);
    if (e != hipSuccess) return;
    Launch<real>::stage_inputs(d, ntr, b->n_in_spikes, dev, s);
    if (forced) Launch<real>::stage_forced(d, ntr, b->n_forced, s);
  };
  // the forward pass in blocks of steps (the tiled kernel delivers step-0 inputs first)
  auto forward = [&]() {
    const uint32_t nblk = (t_max + n->blk - 1) / n->blk;
    // (the no-allocation call instantiates no graph: without one it launches the blocks kernel by kernel)
    if (n->use_graph && !(noalloc && !n->gexec[forced ? 1 : 0])) {
      if (e == hipSuccess) e = ensure_graph(n, d, forced);
      for (uint32_t i = 0; i < nblk && e == hipSuccess; ++i) e = hipGraphLaunch(n->gexec[forced ? 1 : 0], s);
    } else {
      for (uint32_t i = 0; i < nblk; ++i) record_block(n, d, forced, s);
    }
  };
  // device time of fn on the stream (best of two runs; setup() first each time)
  auto timed = [&](auto setup, auto fn) {
    float best = 1e30f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
      setup();
      if (n->use_graph && e == hipSuccess) e = ensure_graph(n, d, forced);  // instantiate outside the timing
      if (e == hipSuccess) e = hipEventRecord(n->tev[0], s);
      fn();
      if (e == hipSuccess) e = hipEventRecord(n->tev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(n->tev[1]);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, n->tev[0], n->tev[1]);
      if (e == hipSuccess && ms < best) best = ms;
    }
    return best;
  };
  const bool tune = !oc && n->autotune_pending && train && !time_driven && !noalloc;

  (void)hipEventRecord(n->ev[0], s);
  // upload
  H2D(n->d_T, b->n_steps, ntr * 4);
  if (b->label) H2D(n->d_label, b->label, ntr * 4);
  if (!dev) {
    H2D(n->d_in_ptr, in_ptr.data(), in_ptr.size() * 8);
    H2D(st_in_step, b->in_step, b->n_in_spikes * 4);
    H2D(st_in_src, b->in_src, b->n_in_spikes * 4);
    const size_t nt = (size_t)ntr * b->step_stride;
    if (b->target) H2D(st_target, b->target, nt * n->K * 8);
    if (b->window) H2D(st_window, b->window, nt);
    if (forced) {
      H2D(n->d_forced_ptr, f_ptr.data(), f_ptr.size() * 8);
      H2D(st_f_step, b->forced_step, b->n_forced * 4);
      H2D(st_f_neuron, b->forced_neuron, b->n_forced * 4);
    }
  }
  restage();
  if (e != hipSuccess) goto device_error;
  if (dev) {
    uint32_t flags = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, d.ctl + eprop::CTL_ERR, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) goto device_error;
    if (flags) {
      set_fail(n, flags & eprop::ERR_INPUT_ORDER ? "input spikes not strictly sorted by (step, source)"
                                                 : "spike out of range");
      return EPROP_ERR_INVALID_ARGUMENT;
    }
  }
  if (oc) {
    const eprop_status ost = run_online(n, d, b, res, *oc, forced, prof, e);
    if (e != hipSuccess) goto device_error;
    return ost;
  }
  if (tune && !n->gather) {
    // Autotuner, part 1: the delivery variant of the forward kernel, then the
    // steps per launch.  Every candidate simulates this batch from rest; the
    // results do not depend on the shapes (FP32 sums are exact fixed point).
    float best = 1e30f;
    uint32_t bv = n->shapes.fwd_variant, bb = n->blk;
    for (uint32_t v = 0; v < eprop::kNumFwdVariants && e == hipSuccess; ++v) {
      if (v == eprop::kQueueVariant && !n->queues) continue;
      n->shapes.fwd_variant = v;
      drop_graphs(n);
      const float ms = timed(restage, forward);
      if (ms < best) { best = ms; bv = v; }
    }
    n->shapes.fwd_variant = bv;
    for (uint32_t blk : {125u, 500u, 1000u}) {
      if (blk > n->Tcap || e != hipSuccess) continue;
      n->blk = blk;
      drop_graphs(n);
      const float ms = timed(restage, forward);
      if (ms < best) { best = ms; bb = blk; }
    }
    n->blk = bb;
    drop_graphs(n);
    restage();
    if (e != hipSuccess) goto device_error;
  }
  if (prof) (void)hipEventRecord(n->ev[1], s);
  forward();
  if (e != hipSuccess) goto device_error;
  if (prof) (void)hipEventRecord(n->ev[2], s);
  // (timed with the readout: the forward phase holds the forward kernel only)
  if (!n->gather) Launch<real>::rec_lists(d, ntr, s);  // the tiled kernel writes bitsets only
  Launch<real>::readout(d, s);
  if (prof) (void)hipEventRecord(n->ev[3], s);
  // the gradient pairs hold nothing yet after an update (or at start): the
  // gradient kernels then write them instead of adding to stale contents
  d.g_fresh = n->trials_accum == 0 ? 1 : 0;
  if (time_driven) {
    Launch<real>::time_driven(d, n->shapes, ntr, static_cast<real *>(n->Lbuf), static_cast<real *>(n->partial), s);
    if (prof) (void)hipEventRecord(n->ev[4], s);
    if (prof) (void)hipEventRecord(n->ev[5], s);
    Launch<real>::output_reduce(d, s);
    if (prof) (void)hipEventRecord(n->ev[6], s);
  } else if (train) {
    if (tune) {
      // part 2: threads per block of the adjoint kernel (idempotent)
      float best = 1e30f;
      uint32_t bbd = n->shapes.adj_block;
      for (uint32_t bd : {64u, 128u, 256u}) {
        if (bd > 64 && n->K > 16) continue;  // LDS of the feedback rows
        n->shapes.adj_block = bd;
        const float ms = timed([] {}, [&] { Launch<real>::adjoint(d, n->shapes, s); });
        if (ms < best) { best = ms; bbd = bd; }
      }
      n->shapes.adj_block = bbd;
    }
    Launch<real>::adjoint(d, n->shapes, s);
    if (prof) (void)hipEventRecord(n->ev[4], s);
    if (tune) {
      // part 3: threads per block and record prefetch depth of the synapse kernel; the accumulators
      // are saved before and restored after every trial run
      void *save = nullptr;
      const size_t gbytes = n->S * sizeof(real);
      if (n->S && dalloc(n, reinterpret_cast<uint8_t **>(&save), 2 * gbytes)) {
        auto keep = [&] {
          if (e == hipSuccess) e = hipMemcpyAsync(save, d.gs, gbytes, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(static_cast<uint8_t *>(save) + gbytes, d.gc, gbytes,
                                                  hipMemcpyDeviceToDevice, s);
        };
        auto back = [&] {
          if (e == hipSuccess) e = hipMemcpyAsync(d.gs, save, gbytes, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(d.gc, static_cast<uint8_t *>(save) + gbytes, gbytes,
                                                  hipMemcpyDeviceToDevice, s);
        };
        keep();
        float best = 1e30f;
        uint32_t bsb = n->shapes.syn_block, bvar = n->shapes.syn_var;
        for (uint32_t var = 0; var < eprop::kNumSynVariants; ++var)
          for (uint32_t sb : {64u, 128u, 256u}) {
            n->shapes.syn_block = sb;
            n->shapes.syn_var = var;
            const float ms = timed(back, [&] {
              Launch<real>::synapse(d, n->shapes, ntr, static_cast<real *>(n->partial), s);
            });
            if (ms < best) { best = ms; bsb = sb; bvar = var; }
          }
        back();
        n->shapes.syn_block = bsb;
        n->shapes.syn_var = bvar;
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        release(n, save);
      }
      n->autotune_pending = false;
      n->tuned = true;
      if (e != hipSuccess) goto device_error;
    }
    Launch<real>::synapse(d, n->shapes, ntr, static_cast<real *>(n->partial), s);
    if (prof) (void)hipEventRecord(n->ev[5], s);
    Launch<real>::output_reduce(d, s);
    if (prof) (void)hipEventRecord(n->ev[6], s);
  }
  (void)hipEventRecord(n->ev[7], s);
  {
    std::vector<double> &loss = n->h_loss;
    std::vector<uint32_t> &pred = n->h_pred;
    loss.resize(ntr);
    pred.resize(ntr);
    unsigned long long cnt[eprop::CNT_WORDS] = {}, ev[64] = {};
    uint32_t flags = 0;
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(loss.data(), d.loss_out, ntr * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(pred.data(), d.pred_out, ntr * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, d.cnt, sizeof(cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ev, d.evcnt, sizeof(ev), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, d.ctl + eprop::CTL_ERR, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) goto device_error;
    n->last_ntr = ntr;
    n->last_T.assign(b->n_steps, b->n_steps + ntr);
    if (flags & eprop::ERR_SYNC) {
      n->failed = true;
      set_fail(n, "spike exchange between the tiles of a trial timed out");
      return EPROP_ERR_DEVICE;
    }
    if (flags & eprop::ERR_INPUT_BOUND) {
      n->failed = true;
      set_fail(n, "weights too large for the FP32 fixed-point input accumulator "
                  "(sum of |w| into one neuron above 2^22)");
      return EPROP_ERR_NUMERIC;
    }
    if (flags) {
      set_fail(n, "forced spike out of range");
      return EPROP_ERR_INVALID_ARGUMENT;
    }
    bool finite_all = true;
    for (uint32_t i = 0; i < ntr; ++i) finite_all = finite_all && std::isfinite(loss[i]);
    if (train) n->trials_accum += ntr;
    if (res) {
      if (res->loss) std::memcpy(res->loss, loss.data(), ntr * 8);
      if (res->predicted) std::memcpy(res->predicted, pred.data(), ntr * 4);
      res->n_rec_spikes = cnt[eprop::CNT_REC_SPIKES];
      res->n_in_spikes = b->n_in_spikes;
      unsigned long long events = 0;
      for (int i = 0; i < 64; ++i) events += ev[i];
      res->n_syn_events = events;
      res->n_out_events = cnt[eprop::CNT_REC_SPIKES] * n->K;
      res->n_eprop_updates = train ? events : 0;
      res->n_flush_updates = train ? cnt[eprop::CNT_FLUSH] : 0;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, n->ev[0], n->ev[7]);
      res->device_seconds = ms * 1e-3;
      for (int p = 0; p < EPROP_N_PHASES; ++p) res->phase_ms[p] = 0;
      if (prof) {
        const int upto = train ? 6 : 3;
        for (int p = 0; p < upto; ++p) {
          float m = 0;
          (void)hipEventElapsedTime(&m, n->ev[p], n->ev[p + 1]);
          res->phase_ms[p] = m;
        }
      }
    }
    if (!finite_all) {
      n->failed = true;
      set_fail(n, "non-finite loss");
      return EPROP_ERR_NUMERIC;
    }
  }
  n->err.clear();
  return EPROP_OK;

device_error:
  n->failed = true;
  set_fail(n, std::string("device error: ") + hip_msg(e));
  return EPROP_ERR_DEVICE;
}

// The e-prop+ schedule over one staged run (trial slot 0 holds the joined
// samples): neuron state, readout and synaptic traces start from rest, the
// weights move to target-major order for the run and back afterwards.
template <typename real>
eprop_status run_online(eprop_network *n, DevNet<real> &d, const eprop_batch *b, eprop_batch_result *res,
                        const OnlineCtx &oc, bool forced, bool prof, hipError_t &e) {
  hipStream_t s = n->stream;
  const uint32_t T = b->n_steps[0], K = n->K, ns = oc.n_samples;
  const size_t T1 = (size_t)n->Tcap + 1;
  const bool ema = n->cfg.reg_mode == EPROP_REG_MOVING_AVERAGE && n->cfg.c_reg != 0.0;
  bool ok = true;
  if (!n->on_syn) {
    uint8_t *p = nullptr;
    ok = dalloc(n, &p, n->S * sizeof(eprop::OnlineSyn<real>));
    n->on_syn = p;
    ok = ok && dalloc(n, &n->on_Eh, T1 * K) && dalloc(n, &n->on_y, K) && dalloc(n, &n->on_zbo, n->Jp) &&
         dalloc(n, &n->on_rdone, n->Jp) && dalloc(n, &n->on_zlast, n->Jp);
    real *pi = nullptr, *pl = nullptr;
    ok = ok && dalloc(n, &pi, n->Jp) && dalloc(n, &pl, T1 * n->Jp);
    n->on_I = pi;
    n->on_L = pl;
  }
  if (ok && ema && !n->on_fh) {
    real *p = nullptr;
    ok = dalloc(n, &p, T1 * n->Jp);
    n->on_fh = p;
  }
  if (ok && !d.tm_w) ok = dalloc(n, &d.tm_w, n->S);
  ok = ok && dgrow(n, &n->on_loss, &n->cap_on_loss, ns) && dgrow(n, &n->on_psum, &n->cap_on_psum, (size_t)ns * K) &&
       dgrow(n, &n->on_off, &n->cap_on_off, ns + 1) && dgrow(n, &n->on_label, &n->cap_on_label, ns);
  if (!ok) {
    set_fail(n, "out of device memory for the online run");
    return EPROP_ERR_OUT_OF_MEMORY;
  }
  auto MS = [&](void *dst, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemsetAsync(dst, 0, bytes, s);
  };
  MS(n->on_syn, n->S * sizeof(eprop::OnlineSyn<real>));
  MS(n->on_Eh, T1 * K * 8);
  MS(n->on_L, T1 * n->Jp * sizeof(real));
  MS(n->on_y, K * 8);
  MS(n->on_zbo, n->Jp * 8);
  MS(n->on_rdone, n->Jp * 4);
  MS(n->on_zlast, n->Jp * 4);
  if (ema) MS(n->on_fh, n->Jp * sizeof(real));  // f at step 0
  MS(n->on_loss, ns * 8);
  MS(n->on_psum, (size_t)ns * K * 8);
  MS(d.psi, n->Jp * sizeof(real));              // psi and spikes at step 0 of trial slot 0
  MS(d.rec_bits, n->Jw * 8);
  if (e == hipSuccess) e = hipMemcpyAsync(n->on_off, oc.off.data(), (ns + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(n->on_label, oc.label.data(), ns * 4, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return EPROP_ERR_DEVICE;
  eprop::OnlineRun<real> o{};
  o.syn = static_cast<eprop::OnlineSyn<real> *>(n->on_syn);
  o.Eh = n->on_Eh;
  o.y = n->on_y;
  o.zbo = n->on_zbo;
  o.r_done = n->on_rdone;
  o.zlast = n->on_zlast;
  o.fh = static_cast<real *>(n->on_fh);
  o.Ibuf = static_cast<real *>(n->on_I);
  o.Lh = static_cast<real *>(n->on_L);
  o.loss = n->on_loss;
  o.psum = n->on_psum;
  o.off = n->on_off;
  o.label = n->on_label;
  o.n_samples = ns;
  o.cutoff = n->cfg.isi_cutoff;
  o.lag = 1 + n->cfg.d_ls + n->cfg.d_out;
  o.eta = n->cfg.eta;
  Launch<real>::online_fill(d, false, s);
  if (prof) (void)hipEventRecord(n->ev[1], s);
  for (uint32_t t = 1; t <= T; ++t) Launch<real>::online_step(d, o, t, forced, s);
  if (prof) (void)hipEventRecord(n->ev[2], s);
  Launch<real>::online_fill(d, true, s);
  if (n->blocked) Launch<real>::input_bound_blocked(d, n->n_ach, s);
  else Launch<real>::input_bound(d, s);
  (void)hipEventRecord(n->ev[7], s);
  std::vector<double> loss(ns), psum((size_t)ns * K);
  unsigned long long cnt[eprop::CNT_WORDS] = {}, ev[64] = {};
  uint32_t flags = 0;
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(loss.data(), n->on_loss, ns * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(psum.data(), n->on_psum, psum.size() * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(cnt, d.cnt, sizeof(cnt), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ev, d.evcnt, sizeof(ev), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, d.ctl + eprop::CTL_ERR, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return EPROP_ERR_DEVICE;
  n->last_ntr = 1;
  n->last_T.assign(1, T);
  if (flags) {
    set_fail(n, "forced spike out of range");
    return EPROP_ERR_INVALID_ARGUMENT;
  }
  bool finite_all = true;
  for (uint32_t c = 0; c < ns; ++c) finite_all = finite_all && std::isfinite(loss[c]);
  if (res) {
    if (res->loss) std::memcpy(res->loss, loss.data(), ns * 8);
    if (res->predicted)
      for (uint32_t c = 0; c < ns; ++c) {
        uint32_t best = 0;
        if (n->cfg.loss != EPROP_LOSS_MSE)
          for (uint32_t k = 1; k < K; ++k)
            if (psum[(size_t)c * K + k] > psum[(size_t)c * K + best]) best = k;
        res->predicted[c] = best;
      }
    res->n_rec_spikes = cnt[eprop::CNT_REC_SPIKES];
    res->n_in_spikes = b->n_in_spikes;
    unsigned long long events = 0;
    for (int i = 0; i < 64; ++i) events += ev[i];
    res->n_syn_events = events;
    res->n_out_events = cnt[eprop::CNT_REC_SPIKES] * K;
    res->n_eprop_updates = events;  // one update per arriving spike
    res->n_flush_updates = 0;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, n->ev[0], n->ev[7]);
    res->device_seconds = ms * 1e-3;
    for (int p = 0; p < EPROP_N_PHASES; ++p) res->phase_ms[p] = 0;
    if (prof) {
      float m = 0;
      (void)hipEventElapsedTime(&m, n->ev[0], n->ev[1]);
      res->phase_ms[0] = m;
      (void)hipEventElapsedTime(&m, n->ev[1], n->ev[2]);
      res->phase_ms[1] = m;  // the whole run is the forward phase
    }
  }
  if (!finite_all) {
    n->failed = true;
    set_fail(n, "non-finite loss");
    return EPROP_ERR_NUMERIC;
  }
  n->err.clear();
  return EPROP_OK;
}

// EPROP_BATCH_ONLINE: validates the samples and joins them into one run.
template <typename real>
eprop_status simulate_online(eprop_network *n, DevNet<real> &d, const eprop_batch *b, eprop_batch_result *res) {
  auto fail = [&](eprop_status st, const char *m) {
    set_fail(n, m);
    return st;
  };
  if (b->flags & ~(uint32_t)(EPROP_BATCH_ONLINE | EPROP_BATCH_TRAIN | EPROP_BATCH_PROFILE | EPROP_RECORD_SPIKES |
                             EPROP_RECORD_TRACES))
    return fail(EPROP_ERR_INVALID_ARGUMENT, "EPROP_BATCH_ONLINE combines only with TRAIN, PROFILE and RECORD_*");
  if (b->memory != EPROP_MEM_HOST) return fail(EPROP_ERR_UNSUPPORTED, "the online schedule takes host-memory batches");
  if (n->cfg.optimizer != EPROP_OPT_GD) return fail(EPROP_ERR_UNSUPPORTED, "the online schedule uses gradient descent");
  if (n->cfg.c_reg != 0.0 && n->cfg.reg_mode == EPROP_REG_STATIC)
    return fail(EPROP_ERR_UNSUPPORTED, "the static rate regulariser needs whole samples; use the moving average");
  if (b->n_trials < 1 || !b->n_steps || !b->in_ptr) return fail(EPROP_ERR_INVALID_ARGUMENT, "empty online batch");
  const uint32_t ns = b->n_trials;
  OnlineCtx oc;
  oc.n_samples = ns;
  oc.off.assign(ns + 1, 0);
  oc.label.assign(ns, 0);
  uint64_t T = 0;
  for (uint32_t c = 0; c < ns; ++c) {
    if (b->n_steps[c] < 1) return fail(EPROP_ERR_INVALID_ARGUMENT, "trial with zero steps");
    T += b->n_steps[c];
    if (T > n->Tcap) return fail(EPROP_ERR_CAPACITY, "the online run is longer than max_steps");
    oc.off[c + 1] = (uint32_t)T;
  }
  const bool cls = n->cfg.loss != EPROP_LOSS_MSE;
  if (cls && !b->label) return fail(EPROP_ERR_INVALID_ARGUMENT, "classification losses need labels");
  if (!cls && !b->target) return fail(EPROP_ERR_INVALID_ARGUMENT, "MSE needs a target");
  if (b->step_stride < 1) return fail(EPROP_ERR_INVALID_ARGUMENT, "step_stride must be >= 1");
  for (uint32_t c = 0; c < ns; ++c) {
    if (b->n_steps[c] > b->step_stride) return fail(EPROP_ERR_INVALID_ARGUMENT, "step_stride smaller than a trial");
    if (cls) {
      if (b->label[c] >= n->K) return fail(EPROP_ERR_INVALID_ARGUMENT, "label out of range");
      oc.label[c] = b->label[c];
    }
  }
  // the joined run: inputs shifted by each sample's offset, targets and
  // windows laid end to end, forced spikes shifted
  std::vector<uint64_t> in_ptr(2, 0), f_ptr(2, 0);
  std::vector<uint32_t> in_step, in_src, f_step, f_neu;
  in_step.reserve(b->n_in_spikes);
  in_src.reserve(b->n_in_spikes);
  for (uint32_t c = 0; c < ns; ++c) {
    const uint64_t lo = b->in_ptr[c], hi = b->in_ptr[c + 1];
    if (hi < lo || hi > b->n_in_spikes) return fail(EPROP_ERR_INVALID_ARGUMENT, "in_ptr out of order");
    for (uint64_t q = lo; q < hi; ++q) {
      if (b->in_step[q] >= b->n_steps[c]) return fail(EPROP_ERR_INVALID_ARGUMENT, "input spike out of its trial");
      in_step.push_back(b->in_step[q] + oc.off[c]);
      in_src.push_back(b->in_src[q]);
    }
    if (b->forced_ptr) {
      for (uint64_t q = b->forced_ptr[c]; q < b->forced_ptr[c + 1]; ++q) {
        if (b->forced_step[q] < 1 || b->forced_step[q] > b->n_steps[c])
          return fail(EPROP_ERR_INVALID_ARGUMENT, "forced spike out of range");
        f_step.push_back(b->forced_step[q] + oc.off[c]);
        f_neu.push_back(b->forced_neuron[q]);
      }
    }
  }
  in_ptr[1] = in_step.size();
  f_ptr[1] = f_step.size();
  std::vector<double> target;
  std::vector<uint8_t> window;
  if (b->target && !cls) {
    target.resize((size_t)T * n->K);
    for (uint32_t c = 0; c < ns; ++c)
      std::memcpy(&target[(size_t)oc.off[c] * n->K], b->target + (size_t)c * b->step_stride * n->K,
                  (size_t)b->n_steps[c] * n->K * 8);
  }
  if (b->window) {
    window.resize(T);
    for (uint32_t c = 0; c < ns; ++c)
      std::memcpy(&window[oc.off[c]], b->window + (size_t)c * b->step_stride, b->n_steps[c]);
  }
  const uint32_t T32 = (uint32_t)T, lab0 = oc.label[0];
  eprop_batch run{};
  run.n_trials = 1;
  run.memory = EPROP_MEM_HOST;
  run.n_steps = &T32;
  run.n_in_spikes = in_step.size();
  run.in_ptr = in_ptr.data();
  run.in_step = in_step.data();
  run.in_src = in_src.data();
  run.step_stride = T32;
  run.target = target.empty() ? nullptr : target.data();
  run.label = cls ? &lab0 : nullptr;
  run.window = window.empty() ? nullptr : window.data();
  if (b->forced_ptr) {
    run.n_forced = f_step.size();
    run.forced_ptr = f_ptr.data();
    run.forced_step = f_step.data();
    run.forced_neuron = f_neu.data();
  }
  run.flags = EPROP_BATCH_TRAIN | (b->flags & EPROP_BATCH_PROFILE);
  return simulate(n, d, &run, res, &oc);
}

template <typename real>
eprop_status apply(eprop_network *n, DevNet<real> &d) {
  const double b1 = n->cfg.adam_beta1, b2 = n->cfg.adam_beta2;
  n->adam_step += 1;
  const double step = (double)n->adam_step;
  // eq. eta-adam-fast
  const double eta_t = n->cfg.eta * std::sqrt(1.0 - std::pow(b2, step)) / (1.0 - std::pow(b1, step));
  if (!n->blocked) {
    Launch<real>::apply(d, n->S, (double)n->trials_accum, n->cfg.optimizer, n->cfg.eta, eta_t, b1, b2,
                        n->cfg.adam_eps_hat, n->stream);
    Launch<real>::input_bound(d, n->stream);
  } else {
    Launch<real>::apply_blocked(d, n->n_ach, n->S, (double)n->trials_accum, n->cfg.optimizer, n->cfg.eta, eta_t,
                                b1, b2, n->cfg.adam_eps_hat, n->stream);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) {
    n->failed = true;
    set_fail(n, std::string("device error: ") + hip_msg(e));
    return EPROP_ERR_DEVICE;
  }
  n->trials_accum = 0;
  n->err.clear();
  return EPROP_OK;
}

template <typename real>
eprop_status read_state(const eprop_network *n, const DevNet<real> &d, int32_t what, uint32_t trial,
                        void *dst, size_t dst_bytes, size_t *needed) {
  const bool per_trial = (what >= EPROP_STATE_SPIKES && what <= EPROP_STATE_V) || what == EPROP_STATE_L;
  if (what < 0 || what > EPROP_STATE_INPUT_BOUND) return EPROP_ERR_INVALID_ARGUMENT;
  if (what == EPROP_STATE_LAYOUT) {
    const uint64_t lay[18] = {d.TS, d.KT, d.ring_bytes, n->shapes.tile_block, n->shapes.syn_block, n->shapes.ginst,
                              n->blk, n->gather ? 1u : 0u, eprop::fwd_variant_piece(n->shapes.fwd_variant),
                              eprop::fwd_variant_unroll(n->shapes.fwd_variant), n->shapes.adj_block,
                              n->tuned ? 1u : 0u, d.ptab_cap, eprop::syn_variant_pre(n->shapes.syn_var),
                              eprop::syn_variant_batch(n->shapes.syn_var), n->blocked ? 1u : 0u,
                              n->shapes.fwd_trials ? n->shapes.fwd_trials : n->Bcap,
                              n->shapes.fwd_variant == eprop::kQueueVariant ? 1u : 0u};
    if (needed) *needed = sizeof(lay);
    if (!dst) return EPROP_OK;
    if (dst_bytes < sizeof(lay)) return EPROP_ERR_INVALID_ARGUMENT;
    std::memcpy(dst, lay, sizeof(lay));
    return EPROP_OK;
  }
  if (per_trial && n->last_ntr == 0) return EPROP_ERR_STATE;
  if (per_trial && trial >= n->last_ntr) return EPROP_ERR_INVALID_ARGUMENT;
  const uint32_t T = per_trial ? n->last_T[trial] : 0;
  const size_t KJ = (size_t)n->K * n->Jp;
  auto fetch = [&](const void *src, size_t count, std::vector<real> &out) {
    out.resize(count);
    return count ? hipMemcpy(out.data(), src, count * sizeof(real), hipMemcpyDeviceToHost) : hipSuccess;
  };
  std::vector<double> outd;
  std::vector<uint32_t> outu;
  uint64_t step = n->adam_step;
  hipError_t e = hipSuccess;
  size_t bytes = 0;
  const void *payload = nullptr;
  switch (what) {
    case EPROP_STATE_INPUT_BOUND: {
      if (!dst) { bytes = 8; break; }
      uint32_t bits = 0;
      e = hipMemcpy(&bits, d.l1max, 4, hipMemcpyDeviceToHost);
      float f;
      std::memcpy(&f, &bits, 4);
      outd.assign(1, (double)f);
      break;
    }
    case EPROP_STATE_W_IN:
    case EPROP_STATE_W_REC: {
      const bool in = what == EPROP_STATE_W_IN;
      if (!dst) { bytes = (in ? n->S_in : n->S_rec) * 8; break; }
      outd.assign(in ? n->S_in : n->S_rec, 0.0);
      auto put = [&](uint32_t o, real w) {
        if ((o < n->S_in) == in) outd[in ? o : o - n->S_in] = (double)w;
      };
      if (!n->blocked) {  // target-major weights, kept by every update
        std::vector<real> w;
        e = fetch(d.tm_w, n->S, w);
        for (uint64_t q = 0; q < n->S && e == hipSuccess; ++q) put(n->perm[q], w[q]);
        break;
      }
      // the delivery table, segment by segment
      const uint32_t KT = d.KT;
      std::vector<uint32_t> dl(n->dl_words), ts((size_t)n->NS * (KT + 1));
      std::vector<uint2> sg((size_t)n->NS * KT);
      e = hipMemcpy(dl.data(), d.dlw, dl.size() * 4, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(ts.data(), d.tseg, ts.size() * 4, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(sg.data(), d.dseg, sg.size() * sizeof(uint2), hipMemcpyDeviceToHost);
      for (uint64_t src = 0; src < n->NS && e == hipSuccess; ++src)
        for (uint32_t k = 0; k < KT; ++k) {
          const uint2 g = sg[src * KT + eprop::tile_rank(k, KT)];
          const real *w = reinterpret_cast<const real *>(dl.data() + g.x);
          const uint32_t q0 = ts[src * (KT + 1) + k];
          for (uint32_t i = 0; i < g.y; ++i) put(n->sm2caller[q0 + i], w[i]);
        }
      break;
    }
    case EPROP_STATE_GRAD_IN: case EPROP_STATE_GRAD_REC:
    case EPROP_STATE_ADAM_M_IN: case EPROP_STATE_ADAM_V_IN:
    case EPROP_STATE_ADAM_M_REC: case EPROP_STATE_ADAM_V_REC: {
      const bool in = what == EPROP_STATE_GRAD_IN || what == EPROP_STATE_ADAM_M_IN || what == EPROP_STATE_ADAM_V_IN;
      const uint64_t cnt = in ? n->S_in : n->S_rec;
      if (!dst) { bytes = cnt * 8; break; }
      if ((what >= EPROP_STATE_ADAM_M_IN) && !n->adam) { outd.assign(cnt, 0.0); break; }
      std::vector<real> a, c;
      if (what == EPROP_STATE_GRAD_IN || what == EPROP_STATE_GRAD_REC) {
        if (n->trials_accum == 0) {  // nothing accumulated since the last update
          outd.assign(cnt, 0.0);
          break;
        }
        e = fetch(d.gs, n->S, a);
        if (e == hipSuccess) e = fetch(d.gc, n->S, c);
      } else {
        const bool m = what == EPROP_STATE_ADAM_M_IN || what == EPROP_STATE_ADAM_M_REC;
        e = fetch(m ? d.adam_m : d.adam_v, n->S, a);
      }
      outd.assign(cnt, 0.0);
      const bool grad = what == EPROP_STATE_GRAD_IN || what == EPROP_STATE_GRAD_REC;
      const std::vector<uint32_t> &ord = (grad || !n->blocked) ? n->perm : n->sm2caller;
      for (uint64_t q = 0; q < n->S && e == hipSuccess; ++q) {
        const uint32_t o = ord[q];
        const bool is_in = o < n->S_in;
        if (is_in != in) continue;
        outd[in ? o : o - n->S_in] = (double)a[q] + (c.empty() ? 0.0 : (double)c[q]);
      }
      break;
    }
    case EPROP_STATE_W_OUT: case EPROP_STATE_GRAD_OUT: case EPROP_STATE_ADAM_M_OUT: case EPROP_STATE_ADAM_V_OUT: {
      if (!dst) { bytes = (size_t)n->K * n->J * 8; break; }
      std::vector<real> a, c;
      if ((what == EPROP_STATE_ADAM_M_OUT || what == EPROP_STATE_ADAM_V_OUT) && !n->adam) {
        outd.assign((size_t)n->K * n->J, 0.0);
        break;
      }
      const real *src = what == EPROP_STATE_W_OUT ? d.w_out : what == EPROP_STATE_GRAD_OUT ? d.gos
                        : what == EPROP_STATE_ADAM_M_OUT ? d.adam_mo : d.adam_vo;
      e = fetch(src, KJ, a);
      if (e == hipSuccess && what == EPROP_STATE_GRAD_OUT) e = fetch(d.goc, KJ, c);
      outd.resize((size_t)n->K * n->J);
      for (uint32_t k = 0; k < n->K; ++k)
        for (uint32_t j = 0; j < n->J; ++j) {
          const size_t i = (size_t)k * n->Jp + j;
          outd[(size_t)k * n->J + j] = (double)a[i] + (c.empty() ? 0.0 : (double)c[i]);
        }
      break;
    }
    case EPROP_STATE_ADAM_STEP:
      bytes = 8;
      payload = &step;
      break;
    case EPROP_STATE_SPIKES: {
      std::vector<uint64_t> bits((size_t)T * n->Jw);
      e = hipMemcpy(bits.data(), d.rec_bits + ((size_t)trial * (n->Tcap + 1) + 1) * n->Jw, bits.size() * 8,
                    hipMemcpyDeviceToHost);
      for (uint32_t t = 1; t <= T && e == hipSuccess; ++t)
        for (uint32_t w = 0; w < n->Jw; ++w) {
          uint64_t word = bits[(size_t)(t - 1) * n->Jw + w];
          while (word) {
            const uint32_t bit = (uint32_t)__builtin_ctzll(word);
            word &= word - 1;
            outu.push_back(t);
            outu.push_back(w * 64 + bit);
          }
        }
      bytes = outu.size() * 4;
      payload = outu.data();
      break;
    }
    case EPROP_STATE_PSI: {
      if (!dst) { bytes = (size_t)T * n->J * 8; break; }
      std::vector<real> a;
      e = fetch(d.psi + ((size_t)trial * (n->Tcap + 1) + 1) * n->Jp, (size_t)T * n->Jp, a);
      outd.resize((size_t)T * n->J);
      for (uint32_t t = 0; t < T && e == hipSuccess; ++t)
        for (uint32_t j = 0; j < n->J; ++j) outd[(size_t)t * n->J + j] = (double)a[(size_t)t * n->Jp + j];
      break;
    }
    case EPROP_STATE_Y: case EPROP_STATE_ERR: {
      bytes = (size_t)T * n->K * 8;
      if (!dst) break;
      outd.resize((size_t)T * n->K);
      const double *src = (what == EPROP_STATE_Y ? d.y : d.err) + ((size_t)trial * (n->Tcap + 2) + 1) * n->K;
      e = hipMemcpy(outd.data(), src, bytes, hipMemcpyDeviceToHost);
      break;
    }
    case EPROP_STATE_L: {  // sum_k B_jk E_k^t in FP64, ascending k
      bytes = (size_t)T * n->J * 8;
      if (!dst) break;
      std::vector<double> err((size_t)T * n->K);
      std::vector<real> fb;
      e = hipMemcpy(err.data(), d.err + ((size_t)trial * (n->Tcap + 2) + 1) * n->K, err.size() * 8,
                    hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = fetch(d.fb, KJ, fb);
      outd.assign((size_t)T * n->J, 0.0);
      for (uint32_t t = 0; t < T && e == hipSuccess; ++t)
        for (uint32_t j = 0; j < n->J; ++j) {
          double acc = 0.0;
          for (uint32_t k = 0; k < n->K; ++k) acc += (double)fb[(size_t)j * n->K + k] * err[(size_t)t * n->K + k];
          outd[(size_t)t * n->J + j] = acc;
        }
      break;
    }
    case EPROP_STATE_V: {
      if (!dst) { bytes = (size_t)n->J * 8; break; }
      std::vector<real> a;
      e = fetch(d.v + (size_t)trial * n->Jp, n->J, a);
      outd.assign(a.begin(), a.end());
      break;
    }
  }
  if (e != hipSuccess) return EPROP_ERR_DEVICE;
  if (!payload && dst) {
    payload = outd.data();
    bytes = outd.size() * 8;
  }
  if (needed) *needed = bytes;
  if (!dst) return EPROP_OK;
  if (dst_bytes < bytes) return EPROP_ERR_INVALID_ARGUMENT;
  if (bytes) std::memcpy(dst, payload, bytes);
  return EPROP_OK;
}

}  // namespace

extern "C" {

eprop_status eprop_simulate_batch(eprop_network *net, const eprop_batch *batch, eprop_batch_result *res) {
  if (!net || !batch) return EPROP_ERR_INVALID_ARGUMENT;
  if (net->failed) return EPROP_ERR_STATE;
  try {
    if (batch->flags & EPROP_BATCH_ONLINE)
      return net->fp64 ? simulate_online(net, net->n64, batch, res) : simulate_online(net, net->n32, batch, res);
    return net->fp64 ? simulate(net, net->n64, batch, res) : simulate(net, net->n32, batch, res);
  } catch (const std::exception &x) {
    set_fail(net, host_failure(x));
  } catch (...) {
    set_fail(net, "host failure");
  }
  // device work of the batch may be half issued: the handle is failed
  (void)hipStreamSynchronize(net->stream);
  net->failed = true;
  return EPROP_ERR_OUT_OF_MEMORY;
}

eprop_status eprop_simulate_batch_noalloc(eprop_network *net, const eprop_batch *batch, eprop_batch_result *res) {
  if (!net || !batch) return EPROP_ERR_INVALID_ARGUMENT;
  if (net->failed) return EPROP_ERR_STATE;
  if (batch->flags & (EPROP_BATCH_ONLINE | EPROP_BATCH_TIME_DRIVEN)) {
    set_fail(net, "eprop_simulate_batch_noalloc runs the event-driven batch schedule only");
    return EPROP_ERR_UNSUPPORTED;
  }
  try {
    return net->fp64 ? simulate(net, net->n64, batch, res, nullptr, true)
                     : simulate(net, net->n32, batch, res, nullptr, true);
  } catch (const std::exception &x) {
    set_fail(net, host_failure(x));
  } catch (...) {
    set_fail(net, "host failure");
  }
  (void)hipStreamSynchronize(net->stream);
  net->failed = true;
  return EPROP_ERR_OUT_OF_MEMORY;
}

eprop_status eprop_apply_updates(eprop_network *net) {
  if (!net) return EPROP_ERR_INVALID_ARGUMENT;
  if (net->failed) return EPROP_ERR_STATE;
  if (net->trials_accum == 0) {
    set_fail(net, "no trials trained since the last update");
    return EPROP_ERR_STATE;
  }
  try {
    return net->fp64 ? apply(net, net->n64) : apply(net, net->n32);
  } catch (const std::exception &x) {
    set_fail(net, host_failure(x));
  } catch (...) {
    set_fail(net, "host failure");
  }
  (void)hipStreamSynchronize(net->stream);
  net->failed = true;
  return EPROP_ERR_OUT_OF_MEMORY;
}

eprop_status eprop_read_state(const eprop_network *net, int32_t what, uint32_t trial, void *dst,
                              size_t dst_bytes, size_t *bytes_needed) {
  if (!net) return EPROP_ERR_INVALID_ARGUMENT;
  try {
    return net->fp64 ? read_state(net, net->n64, what, trial, dst, dst_bytes, bytes_needed)
                     : read_state(net, net->n32, what, trial, dst, dst_bytes, bytes_needed);
  } catch (...) {
    // (reading changes nothing on the handle; only the host copy failed)
    return EPROP_ERR_OUT_OF_MEMORY;
  }
}

}  // extern "C"
