// Host runtime and C ABI of libabm: parameter and population validation, workspace
// layout, per-run tables (Gamma infectiousness integral of eq. 1, Poisson thresholds,
// vaccination priority classes of Table 1), the HIP-graph day loop, and the adjoint
// driver of the relaxed (soft) mode.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "abm_internal.h"

using namespace abm;

namespace {

// ---- tables --------------------------------------------------------------------------
// Regularised lower incomplete gamma P(a, x) from its power series
//   P(a, x) = x^a e^-x sum_n x^n / Gamma(a + n + 1).
double gamma_lower_reg(double a, double x) {
  if (x <= 0.0) return 0.0;
  double term = std::exp(a * std::log(x) - x - std::lgamma(a + 1.0));
  double sum = term;
  for (int n = 1; n < 100000; ++n) {
    term *= x / (a + n);
    sum += term;
    if (term < 1e-18 * sum && n > x) break;
  }
  return std::min(sum, 1.0);
}

// Atab[tau] = A_{stage(tau)} * integral of the Gamma(shape, scale) density over the
// day [tau - 1, tau] since exposure; exposed for tau <= e_days, infected until
// e_days + i_days, nothing afterwards (eq. 1).
void build_atab(const abm_params& p, float* out) {
  for (int t = 0; t < ATAB; ++t) out[t] = 0.f;
  for (int t = 1; t <= p.e_days + p.i_days; ++t) {
    const double ph = gamma_lower_reg(p.gamma_shape, t / p.gamma_scale) -
                      gamma_lower_reg(p.gamma_shape, (t - 1) / p.gamma_scale);
    const double A = t <= p.e_days ? p.A_stage[ABM_STAGE_E] : p.A_stage[ABM_STAGE_I];
    out[t] = (float)(A * ph);
  }
}

// The course: Atab[16 c + tau] = A_c * Phi(tau) for the infectious classes c = 1
// (asymptomatic, A_asym), 2 (presymptomatic, A_stage[E]), 3 (symptomatic, A_stage[I])
// and 1 <= tau <= 15; hospitalised agents are isolated.
void build_atab_course(const abm_params& p, float* out) {
  for (int t = 0; t < ATAB; ++t) out[t] = 0.f;
  const double A[4] = {0.0, p.A_asym, p.A_stage[ABM_STAGE_E], p.A_stage[ABM_STAGE_I]};
  for (int c = 1; c <= 3; ++c)
    for (int t = 1; t <= 15; ++t) {
      const double ph = gamma_lower_reg(p.gamma_shape, t / p.gamma_scale) -
                        gamma_lower_reg(p.gamma_shape, (t - 1) / p.gamma_scale);
      out[16 * c + t] = (float)(A[c] * ph);
    }
}

// Poisson(m) inverse-CDF thresholds: T_k = min(floor(F_k 2^32), 2^32 - 1), with the CDF
// accumulated left to right from pmf_0 = e^-m, pmf_k = pmf_{k-1} m / k.
void build_poisson(double m, uint32_t* T) {
  double pmf = std::exp(-m), F = pmf;
  for (int k = 0; k < 64; ++k) {
    if (k) {
      pmf = pmf * m / k;
      F = F + pmf;
    }
    const double v = std::floor(F * 4294967296.0);
    T[k] = v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
  }
}

// Priority class (0 = first) of (dose, age group) under a strategy of Table 1.
int priority_class(int strategy, int dose, int age) {
  switch (strategy) {
    case ABM_STRATEGY_STANDARD: return (dose == 2 ? 0 : 9) + (8 - age);
    case ABM_STRATEGY_DELAYED: return (dose == 1 ? 0 : 9) + (8 - age);
    default:
      if (age >= 6) return 2 * (8 - age) + (dose == 1 ? 0 : 1);
      return 6 + (dose == 1 ? 0 : 6) + (5 - age);
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t total = 0;
  template <typename T>
  size_t take(size_t n) {
    const size_t off = total;
    total = align_up(total + n * sizeof(T));
    return off;
  }
};

struct Offsets {
  size_t rep, tiles, srec, age, hhn, wpm, atab, ptab, dtab, state, code, imask, cmask, scmask, lambda, own, recv, row_ptr,
      cur_occ, cur_rand, col, scan_part, vhist, vplan, vtile, latch, vpart, vsegbase, tile_counts, fin_part, prev_counts,
      traj, day, flags, seeds, ring_rp, ring_col, den_mask, rmask, ninf, work, nwork;
  size_t pb_hist1, pb_own, pb_tbase, pb_part, pb_bstart, pb_bchunk, pb_nchunks, pb_chunks, pb_hist2, pb_leaf, pb_b1h,
      pb_b1w, pb_buf2, pb_tdeg, pb_tstart, pb_tpart;
  size_t s, ehist, inf, sigma, soft_inc, seg_sigma, seg_y, seg_s, ckpt, s_bar, ibar, vtmp, lam_bar,
      gtheta, gpart, dL;
};

struct Sizes {
  int64_t N = 0, R = 0, ntiles = 0, nscan = 0, M = 0, nseeds = 0, ecap = 0, T = 0;
  int64_t seg = 0, nckpt = 0;
  // partitioned builder
  int64_t pb_on = 0, lb = 0, nlv = 0, nb1 = 0, nbatch = 0, bpw = 1, ngrid = 0, bcap = 0, s1_nparts = 0, maxch = 0, nleaf = 0, ccap = 0;
  int64_t asm_cap = 0, s1_cap = PB_S1_CAP, rper = 12;
  int64_t fseg = 1, fin_one = 0, vseg = 0;
};

// element strides of the notification ring's slots, rounded to 64 elements so that
// every slot starts on a 256-byte boundary (the message kernel reads 16-byte groups)
int64_t ring_rstride(const Sizes& z) { return (z.N + 1 + 63) & ~(int64_t)63; }
int64_t ring_cstride(const Sizes& z) { return (z.ecap + 63) & ~(int64_t)63; }
// graph slots: the notification window; in relaxed mode every day of the run if their
// graphs fit in 16 GB (built once by the forward pass, reused by the adjoint's recompute
// and reverse sweep and by later runs at new parameters), else the checkpoint interval
// (a segment's graphs are built by its recompute and reused by the reverse sweep), else
// one slot (every use builds the graph)
constexpr double RING_BUDGET = 16e9;
int64_t ring_slots(const Sizes& z, const abm_params& p) {
  if (p.app_adoption > 0.f) return p.den_window;
  if (p.mode == ABM_SOFT) {
    const double slot = (double)(ring_rstride(z) + ring_cstride(z)) * 4.0;
    if (z.T > 1 && (double)z.T * slot <= RING_BUDGET) return z.T;
    if (z.seg > 1 && (double)z.seg * slot <= RING_BUDGET) return z.seg;
  }
  return 1;
}
// room of one list of flagged rows.  List b takes the 256-agent groups g with
// g mod FRONT_NB = b: at most ceil(ceil(N/256)/FRONT_NB) groups of 256, and there are
// at least ceil(N/256) tiles, so this bound holds
int64_t front_cap(const Sizes& z) { return (z.ntiles + FRONT_NB - 1) / FRONT_NB * TILE; }

}  // namespace

struct abm_sim {
  abm_params p{};
  Sizes z;
  Offsets o{};
  Dev d{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  // one day graph, or one per ring slot when the day's graph is built into the
  // notification ring (the slot is baked into the captured kernel arguments)
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  int err = ABM_OK;
  std::string msg;
  int32_t host_day = 0;
  bool soft_ready = false;
  // relaxed mode with a graph slot for every day: graphs of days [0, graphs_built) are
  // in their slots (a day's graph depends on the seed, stream words and day only, so
  // new parameters from abm_set_theta keep them valid)
  int32_t graphs_built = 0;
  std::vector<RepInfo> reps;
  char* ws = nullptr;
  // profiling: one set of nk + 1 events per day enqueued since the last read-out
  int nk = 0;
  std::vector<std::string> names;
  std::vector<std::vector<hipEvent_t>> prof_sets;
  size_t prof_used = 0;
  std::vector<double> ms;
  std::vector<int64_t> launches;

  int fail(int code, const char* fmt, ...) {
    if (err == ABM_OK) {
      char buf[512];
      va_list ap;
      va_start(ap, fmt);
      vsnprintf(buf, sizeof buf, fmt, ap);
      va_end(ap);
      err = code;
      msg = buf;
    }
    return err;
  }
};


#define HIPCHK(s, x)                                                              \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) return (s)->fail(ABM_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

namespace {

int validate(const abm_params* p, const abm_population* pop, Sizes& z, std::string& why) {
  auto bad = [&](const char* w) {
    why = w;
    return ABM_E_ARG;
  };
  if (!p || !pop) return bad("null params or population");
  if (p->struct_size != sizeof(abm_params) || p->abi_version != ABM_ABI_VERSION) {
    why = "abm_params struct_size/abi_version mismatch";
    return ABM_E_ABI;
  }
  if (pop->n_replicates < 1) return bad("n_replicates < 1");
  if (!pop->agent_offset || !pop->age || !pop->hh_start || !pop->occupation || !pop->R ||
      !pop->susceptibility || !pop->dose2_delay || !pop->init_offset)
    return bad("missing population array");
  if (p->n_steps < 1 || p->n_steps > 32000) return bad("n_steps out of range [1, 32000]");
  if (p->mode != ABM_HARD && p->mode != ABM_SOFT) return bad("mode");
  if (!(p->dt > 0.f)) return bad("dt <= 0");
  if (p->e_days < 1 || p->i_days < 1 || p->e_days + p->i_days > ATAB - 1 ||
      p->e_days + p->i_days >= WIN)
    return bad("e_days/i_days out of range (sum <= 15)");
  if (!(p->gamma_shape > 0) || !(p->gamma_scale > 0)) return bad("gamma parameters");
  for (int k = 0; k < ABM_N_AGE; ++k)
    if (!(p->mu_random[k] >= 0 && p->mu_random[k] <= 40)) return bad("mu_random out of [0, 40]");
  for (int k = 0; k < ABM_N_OCC; ++k)
    if (!(p->mu_occupation[k] >= 0 && p->mu_occupation[k] <= 40)) return bad("mu_occupation out of [0, 40]");
  if (p->test_rate > 0.f && p->test_delay < 1) return bad("test_delay must be >= 1");
  if (p->test_delay_max < p->test_delay || p->test_delay_max > 30)
    return bad("test_delay_max must be in [test_delay, 30]");
  if (!(p->app_adoption >= 0.f && p->app_adoption <= 1.f)) return bad("app_adoption out of [0, 1]");
  if (!(p->den_compliance >= 0.f && p->den_compliance <= 1.f)) return bad("den_compliance out of [0, 1]");
  if (p->app_adoption > 0.f) {
    if (p->mode != ABM_HARD) return bad("exposure notification runs in hard mode only");
    if (p->den_window < 1 || p->den_window > 30) return bad("den_window out of [1, 30]");
    if (p->test_delay < 1) return bad("test_delay must be >= 1");
  }
  if (p->quarantine_days < 0 || p->quarantine_days > 10000) return bad("quarantine_days");
  // day fields of the agent record are int16: the last quarantine must end in range
  // (stage ends of the course come at most 60 + 63 days after their start)
  if (p->n_steps + p->quarantine_days > 32767) return bad("n_steps + quarantine_days > 32767");
  if (p->dose_lag < 0 || p->dose_lag > 10000) return bad("dose_lag");
  if (p->strategy < 0 || p->strategy > 2) return bad("strategy");
  if (!(p->vacc_rate >= 0 && p->vacc_rate <= 1)) return bad("vacc_rate");
  if ((p->flags & ABM_FLAG_STRAIGHT_THROUGH) && p->mode != ABM_SOFT)
    return bad("the straight-through estimator is a relaxed-mode option");
  if (p->mode == ABM_SOFT) {
    if (!(p->gumbel_tau > 0.f)) return bad("gumbel_tau <= 0");
    if (p->checkpoint_every < 1) return bad("checkpoint_every < 1");
  }
  if (p->disease_model != ABM_DISEASE_SEIRM && p->disease_model != ABM_DISEASE_COURSE)
    return bad("disease_model");
  if (p->vacc_immunity != ABM_IMMUNITY_STERILISING && p->vacc_immunity != ABM_IMMUNITY_ASYMPTOMATIC)
    return bad("vacc_immunity");
  if (p->vacc_immunity == ABM_IMMUNITY_ASYMPTOMATIC && p->disease_model != ABM_DISEASE_COURSE)
    return bad("asymptomatic vaccine immunity needs the eleven-stage course");
  if (p->disease_model == ABM_DISEASE_COURSE) {
    if (p->mode != ABM_HARD) return bad("the eleven-stage course runs in hard mode only");
    const float* tabs[5] = {p->p_asym, p->p_severe, p->p_hosp, p->p_icu, p->p_die};
    for (const float* t : tabs)
      for (int a = 0; a < ABM_N_AGE; ++a)
        if (!(t[a] >= 0.f && t[a] <= 1.f)) return bad("course probability out of [0, 1]");
    if (!(p->A_asym >= 0)) return bad("A_asym < 0");
    for (int k = 0; k < ABM_N_DUR; ++k) {
      if (p->dur_shift[k] < 1 || p->dur_shift[k] > 60) return bad("dur_shift out of [1, 60]");
      if (!(p->dur_extra[k] >= 0 && p->dur_extra[k] <= 20)) return bad("dur_extra out of [0, 20]");
    }
  }
  const int R = pop->n_replicates;
  if (pop->agent_offset[0] != 0) return bad("agent_offset[0] != 0");
  for (int r = 0; r < R; ++r)
    if (pop->agent_offset[r + 1] <= pop->agent_offset[r]) return bad("empty or decreasing replicate");
  const int64_t N = pop->agent_offset[R];
  if (N >= (int64_t)1 << 30) return bad("more than 2^30 - 1 agents");   // 30-bit column agent ids
  z.N = N;
  z.R = R;
  z.T = p->n_steps;
  for (int64_t i = 0; i < N; ++i) {
    if (pop->age[i] >= ABM_N_AGE) return bad("age group out of range");
    if (pop->occupation[i] >= ABM_N_OCC) return bad("occupation out of range");
  }
  if (pop->n_households < 1 || pop->hh_start[0] != 0 || pop->hh_start[pop->n_households] != N)
    return bad("hh_start must run from 0 to N");
  {
    int r = 0;
    for (int h = 0; h < pop->n_households; ++h) {
      const int64_t a = pop->hh_start[h], b = pop->hh_start[h + 1];
      if (b <= a || b - a > 255) return bad("household size must be 1..255");
      while (a >= pop->agent_offset[r + 1]) ++r;
      if (b > pop->agent_offset[r + 1]) return bad("household crosses a replicate boundary");
    }
  }
  if (pop->n_workplaces < 0) return bad("n_workplaces < 0");
  if (pop->n_workplaces > 0) {
    if (!pop->wp_start || !pop->wp_members) return bad("missing workplace arrays");
    if (pop->wp_start[0] != 0) return bad("wp_start[0] != 0");
    for (int w = 0; w < pop->n_workplaces; ++w) {
      const int64_t m = (int64_t)pop->wp_start[w + 1] - pop->wp_start[w];
      if (m < 1 || m > 65535) return bad("workplace size must be 1..65535");
    }
    z.M = pop->wp_start[pop->n_workplaces];
  }
  for (int r = 0; r < R; ++r) {
    if (!(pop->R[r] >= 0.f) || !std::isfinite(pop->R[r])) return bad("R must be finite >= 0");
    for (int a = 0; a < ABM_N_AGE; ++a)
      if (!(pop->susceptibility[r * ABM_N_AGE + a] >= 0.f) ||
          !std::isfinite(pop->susceptibility[r * ABM_N_AGE + a]))
        return bad("susceptibility must be finite >= 0");
    if (pop->dose2_delay[r] < 0 || pop->dose2_delay[r] > 10000) return bad("dose2_delay");
    if (pop->init_offset[r + 1] < pop->init_offset[r]) return bad("init_offset decreasing");
  }
  if (pop->init_offset[0] != 0) return bad("init_offset[0] != 0");
  z.nseeds = pop->init_offset[R];
  if (z.nseeds > 0 && !pop->initial_infected) return bad("missing initial_infected");
  for (int r = 0; r < R; ++r)
    for (int64_t k = pop->init_offset[r]; k < pop->init_offset[r + 1]; ++k) {
      const int64_t i = pop->initial_infected[k];
      if (i < pop->agent_offset[r] || i >= pop->agent_offset[r + 1])
        return bad("initial infection outside its replicate");
    }
  z.ntiles = 0;
  int64_t max_rep_tiles = 0;
  for (int r = 0; r < R; ++r) {
    const int64_t nt = (pop->agent_offset[r + 1] - pop->agent_offset[r] + TILE - 1) / TILE;
    z.ntiles += nt;
    max_rep_tiles = std::max(max_rep_tiles, nt);
  }
  // end-of-day count reduction: each replicate's tile rows in fseg parts of 256 lanes
  z.fseg = std::max<int64_t>(1, std::min<int64_t>(256, (max_rep_tiles + 255) / 256));
  // up to 2048 tiles a replicate, one launch reduces and closes the day
  z.fin_one = max_rep_tiles <= 2048;
  // vaccination plan: above 2048 tiles a replicate, its tiles are summed and ranked in
  // segments of 256 by their own workgroups
  z.vseg = (max_rep_tiles <= 2048 && !(p->flags & ABM_FLAG_SEGMENT_VPLAN)) ? 0 : (max_rep_tiles + 255) / 256;
  z.nscan = (N + SCAN_BLOCK - 1) / SCAN_BLOCK;
  // Edge room: mean directed edges + 8 standard deviations of the Poisson contact count.
  double hh_edges = 0;
  for (int h = 0; h < pop->n_households; ++h) {
    const double s = (double)pop->hh_start[h + 1] - pop->hh_start[h];
    hh_edges += s * (s - 1);
  }
  std::vector<uint16_t> wpn(N, 0);
  // replicates are separate populations: a workplace's members share one (the graph
  // builder numbers a partner within its initiator's replicate)
  const int64_t* ao = pop->agent_offset;
  auto rep_of = [&](int64_t a) { return (int64_t)(std::upper_bound(ao, ao + R + 1, a) - ao) - 1; };
  for (int w = 0; w < pop->n_workplaces; ++w) {
    int64_t rw = -1;
    for (int64_t q = pop->wp_start[w]; q < pop->wp_start[w + 1]; ++q) {
      const int64_t a = pop->wp_members[q];
      if (a < 0 || a >= N) return bad("workplace member out of range");
      if (q == pop->wp_start[w]) rw = rep_of(a);
      else if (a < ao[rw] || a >= ao[rw + 1]) return bad("workplace crosses a replicate boundary");
      wpn[a] = (uint16_t)(pop->wp_start[w + 1] - pop->wp_start[w]);
    }
  }
  double cmean = 0;
  for (int r = 0; r < R; ++r) {
    const int64_t lo = pop->agent_offset[r], hi = pop->agent_offset[r + 1];
    for (int64_t i = lo; i < hi; ++i) {
      if (wpn[i] >= 2) cmean += p->mu_occupation[pop->occupation[i]] / 2.0;
      if (hi - lo >= 2) cmean += p->mu_random[pop->age[i]] / 2.0;
    }
  }
  const double emean = hh_edges + 2 * cmean;
  const double ecap = p->edge_capacity > 0 ? (double)p->edge_capacity
                                           : std::ceil(emean + 8.0 * 2.0 * std::sqrt(cmean) + 4096.0);
  if (ecap >= 2147483000.0) {
    why = "planned edge room exceeds int32 row pointers";
    return ABM_E_CAPACITY;
  }
  z.ecap = (int64_t)ecap;
  // room for the day's contacts: at least what the edge room leaves after the household
  // edges (each contact is two edges), so that a larger edge_capacity enlarges both
  z.ccap = (int64_t)std::ceil(std::max(cmean + 8.0 * std::sqrt(cmean), (ecap - hh_edges) / 2.0) + 4096.0);
  // partitioned builder geometry: destinations numbered by tile slot, leaves of 2^lb
  // slots (one tile, or two where one-tile leaves would make more than 512 level-1
  // buckets), level-1 buckets of 256 leaves
  const int64_t slots = z.ntiles * TILE;
  auto nb1_of = [&](int b) { return (slots + ((int64_t)1 << (b + 8)) - 1) >> (b + 8); };
  z.lb = (nb1_of(8) > 512 || (p->flags & ABM_FLAG_TWO_TILE_LEAVES)) ? 9 : 8;
  z.nb1 = nb1_of((int)z.lb);
  z.nlv = (z.ntiles + ((int64_t)1 << (z.lb - 8)) - 1) >> (z.lb - 8);
  // room for a batch's own draws: 1.3x the largest per-agent Poisson means (+2048);
  // the generation pass stages a batch in LDS, so more than 24576 draws (high contact
  // means) take the claim builder
  double mo = 0, mr = 0;
  for (int k = 0; k < ABM_N_OCC; ++k) mo = std::max(mo, p->mu_occupation[k] / 2.0);
  for (int k = 0; k < ABM_N_AGE; ++k) mr = std::max(mr, p->mu_random[k] / 2.0);
  z.bcap = ((int64_t)(1.3 * 1024.0 * (mo + mr)) + 2048 + 255) / 256 * 256;
  z.pb_on = !(p->flags & ABM_FLAG_CLAIM_BUILDER) && z.nb1 <= 1024 &&
            z.ccap < ((int64_t)1 << 31) && z.bcap <= 24576 &&
            N < ((int64_t)1 << 27);   // initiators fit the 27 low bits of a partition word
  // edges of a leaf staged in LDS by the row pass: 1.1x the mean (+512), at most 64 KB
  const double leaf_mean = emean * (double)((int64_t)1 << z.lb) / (double)N;
  z.asm_cap = std::max<int64_t>(2048, std::min<int64_t>(16384, ((int64_t)(1.1 * leaf_mean) + 512 + 255) / 256 * 256));
  if (p->flags & ABM_FLAG_MIN_LDS_ROOM) {
    z.asm_cap = 2048;
    z.s1_cap = 0;
    z.rper = 1;
  }
  z.nbatch = (z.ntiles + 3) / 4;
  // batches per generation / level-1 workgroup: up to 16, keeping >= 1024 workgroups
  z.bpw = std::max<int64_t>(1, std::min<int64_t>(16, z.nbatch / 1024));
  // a level-1 workgroup keeps its batches' run offsets in LDS
  z.bpw = std::max<int64_t>(1, std::min<int64_t>(z.bpw, PB_HS_MAX / std::max<int64_t>(z.nb1, 1) - 1));
  z.ngrid = (z.nbatch + z.bpw - 1) / z.bpw;
  z.s1_nparts = (z.nb1 * z.nbatch + SCAN_BLOCK - 1) / SCAN_BLOCK;
  z.maxch = (z.ccap + 8191) / 8192 + z.nb1;
  z.nleaf = z.nb1 << 8;
  if (p->mode == ABM_SOFT) {
    z.seg = p->checkpoint_every;
    z.nckpt = (z.T + z.seg - 1) / z.seg + 1;
  }
  return ABM_OK;
}

void layout(const Sizes& z, const abm_params& p, Offsets& o, size_t& total) {
  Layout L;
  o.rep = L.take<RepInfo>(z.R);
  o.tiles = L.take<int4>(z.ntiles);
  o.srec = L.take<StaticRec>(z.N);
  o.age = L.take<uint8_t>(z.N);
  o.hhn = L.take<uint8_t>(z.N);
  o.wpm = L.take<int32_t>(std::max<int64_t>(z.M, 1));
  o.atab = L.take<float>(ATAB);
  o.ptab = L.take<uint32_t>(NPT * 64);
  o.dtab = L.take<uint32_t>(ABM_N_DUR * 64);
  o.state = L.take<AgentState>(z.N);
  o.code = L.take<uint8_t>(z.N + 32);
  o.imask = L.take<uint32_t>((z.N + 255) / 256 * 8 + 8);
  o.cmask = L.take<uint32_t>((z.N + 255) / 256 + 1);
  o.scmask = L.take<unsigned long long>((z.N + 16383) / 16384 + 4);
  o.lambda = L.take<float>(z.N);
  o.own = L.take<uint16_t>(z.N);
  o.recv = L.take<uint32_t>(z.N);
  const int64_t nring = ring_slots(z, p);
  if (nring == 1) o.row_ptr = L.take<int32_t>(z.N + 1);
  o.cur_occ = L.take<int32_t>(z.N);
  o.cur_rand = L.take<int32_t>(z.N);
  if (nring == 1) o.col = L.take<int32_t>(z.ecap + 4);    // +4: the message kernel reads 16-byte groups
  o.scan_part = L.take<int64_t>(z.nscan + 1);
  o.vhist = L.take<int32_t>(z.ntiles * NBUCKET);
  o.vplan = L.take<int32_t>(2 * z.R);
  o.vtile = L.take<int32_t>(z.ntiles);
  o.latch = L.take<uint8_t>(z.R);
  if (z.vseg) {
    o.vpart = L.take<int32_t>(z.R * z.vseg * NBUCKET);
    o.vsegbase = L.take<int32_t>(z.R * z.vseg);
  }
  o.tile_counts = L.take<uint32_t>(z.ntiles * TILE_NC);
  o.fin_part = L.take<unsigned long long>(z.R * z.fseg * TILE_NC);
  o.prev_counts = L.take<long long>(z.R * ABM_NC);
  o.traj = L.take<long long>(z.T * z.R * ABM_NC);
  o.day = L.take<int32_t>(2);                  // the day, and the count of replicates done with it
  o.rmask = L.take<uint32_t>((z.N + 31) / 32 + 1);
  o.ninf = L.take<int32_t>(1);
  o.work = L.take<int32_t>((int64_t)FRONT_NB * front_cap(z));
  o.nwork = L.take<int32_t>(FRONT_NB);
  if (nring > 1) {
    // the day's graph lives in slot day % nring; slots start on 256-byte bounds
    o.ring_rp = L.take<int32_t>(nring * ring_rstride(z));
    o.ring_col = L.take<int32_t>(nring * ring_cstride(z) + 4);
  }
  if (p.app_adoption > 0.f) o.den_mask = L.take<uint32_t>((z.N + 31) / 32 + 1);
  o.flags = L.take<int32_t>(1);
  o.seeds = L.take<int32_t>(std::max<int64_t>(z.nseeds, 1));
  if (z.pb_on) {
    o.pb_hist1 = L.take<int32_t>(z.nbatch * z.nb1 + 1);
    o.pb_own = L.take<uint32_t>(z.nbatch * z.bcap);
    o.pb_tbase = L.take<int2>(z.ntiles);
    o.pb_part = L.take<int64_t>(z.s1_nparts + 1);
    o.pb_bstart = L.take<int32_t>(z.nb1 + 1);
    o.pb_bchunk = L.take<int32_t>(z.nb1 + 1);
    o.pb_nchunks = L.take<int32_t>(1);
    o.pb_chunks = L.take<int4>(z.maxch);
    o.pb_hist2 = L.take<int32_t>(z.maxch * 256);
    o.pb_leaf = L.take<int32_t>(z.nleaf + 1);
    o.pb_b1h = L.take<uint16_t>(z.ccap);
    o.pb_b1w = L.take<uint32_t>(z.ccap);
    o.pb_buf2 = L.take<uint2>(z.ccap);
    o.pb_tdeg = L.take<int32_t>(z.ntiles);
    o.pb_tstart = L.take<int32_t>(z.nlv);
    o.pb_tpart = L.take<int64_t>((z.nlv + 1023) / 1024 + 1);
  }
  if (p.mode == ABM_SOFT) {
    o.s = L.take<float>(z.N);
    o.ehist = L.take<float>(WIN * z.N);
    o.inf = L.take<float>(z.N);
    o.sigma = L.take<float>(z.N);
    o.soft_inc = L.take<float>(z.R * z.T);
    o.seg_sigma = L.take<float>(z.seg * z.N);
    o.seg_y = L.take<float>(z.seg * z.N);
    o.seg_s = L.take<float>(z.seg * z.N);
    o.ckpt = L.take<float>(z.nckpt * (WIN + 1) * z.N);
    o.s_bar = L.take<float>(z.N);
    o.ibar = L.take<float>(WIN * z.N);
    o.vtmp = L.take<float>(z.N);
    o.lam_bar = L.take<float>(z.N);
    o.gtheta = L.take<float>(z.R * ABM_N_THETA);
    o.gpart = L.take<float>(z.ntiles * ABM_N_THETA);
    o.dL = L.take<float>(z.R * z.T);
  }
  total = L.total;
}

// The day's kernel chain: interventions, graph build (named steps), force of
// infection, fused step, bookkeeping.  With `ev`, an event is recorded before every
// named step and after the last one.
// The kernel arguments of day `day`.  With exposure notification on, that day's graph
// (row pointers and columns) is built straight into ring slot day % den_window, where
// the pre-pass of the following den_window days reads it: no copy.
Dev day_dev(const abm_sim* s, int64_t day) {
  Dev d = s->d;
  if (d.ring_n > 1) {
    const int64_t slot = day % d.ring_n;
    d.row_ptr = d.ring_rp + slot * d.ring_rstride;
    d.col = d.ring_col + slot * d.ring_cstride;
  }
  return d;
}

void enqueue_day(abm_sim* s, int64_t day, hipStream_t st, const std::vector<hipEvent_t>* ev) {
  const Dev d = day_dev(s, day);
  int k = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord((*ev)[k], st);
    ++k;
  };
  mark();
  launch_pre(d, st);
  mark();
  launch_mask(d, st);
  mark();
  if (d.vacc_on) launch_vplan(d, st);
  for (int b = 0; b < build_steps(d); ++b) {
    mark();
    launch_build_step(d, b, st);
  }
  mark();
  launch_message(d, st);
  mark();
  launch_fused(d, st);
  mark();
  launch_finalize(d, st);
  if (d.den_on) launch_den_clear(d, st);
  if (ev) (void)hipEventRecord((*ev)[k], st);
}

void name_kernels(abm_sim* s) {
  s->names = {"pre", "mask", "vplan"};
  for (int b = 0; b < build_steps(s->d); ++b) s->names.push_back(build_step_name(s->d, b));
  for (const char* n : {"message", "fused", "finalize"}) s->names.push_back(n);
  s->nk = (int)s->names.size();
  s->ms.assign(s->nk, 0.0);
  s->launches.assign(s->nk, 0);
}

// Accumulate the per-kernel times of every profiled day enqueued so far.
int drain_profile(abm_sim* s) {
  if (s->prof_used == 0) return ABM_OK;
  HIPCHK(s, hipStreamSynchronize(s->stream));
  for (size_t q = 0; q < s->prof_used; ++q) {
    const std::vector<hipEvent_t>& ev = s->prof_sets[q];
    for (int k = 0; k < s->nk; ++k) {
      float ms = 0.f;
      HIPCHK(s, hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      s->ms[k] += ms;
      s->launches[k] += 1;
    }
  }
  s->prof_used = 0;
  return ABM_OK;
}

// Autotuner: time every message-kernel variant (LDS chunk x grid shape) on day 0's
// graph and keep the fastest.  Every variant sums each row in the same order, so the
// choice changes timing only.  Day 0's pre-pass and graph build leave the agent state
// untouched (no result is due and nobody is quarantined before day 0).
int autotune(abm_sim* s) {
  Dev& d = s->d;
  hipStream_t st = s->stream;
  launch_pre(d, st);
  launch_mask(d, st);
  for (int b = 0; b < build_steps(d); ++b) launch_build_step(d, b, st);
  hipEvent_t e0, e1;
  HIPCHK(s, hipEventCreate(&e0));
  HIPCHK(s, hipEventCreate(&e1));
  float best = 1e30f;
  int32_t best_chunk = d.msg_chunk, best_grid = d.msg_grid, best_shape = d.msg_shape;
  const int32_t sparse_div = d.sparse_div;
  d.sparse_div = 0;                                        // the streaming kernels run
  for (int v = 0; v < message_variants(); ++v) {
    message_variant(d, v, &d.msg_chunk, &d.msg_grid, &d.msg_shape);
    launch_message(d, st);                                 // warm-up
    HIPCHK(s, hipEventRecord(e0, st));
    for (int rep = 0; rep < 3; ++rep) launch_message(d, st);
    HIPCHK(s, hipEventRecord(e1, st));
    HIPCHK(s, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_chunk = d.msg_chunk;
      best_grid = d.msg_grid;
      best_shape = d.msg_shape;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  d.msg_chunk = best_chunk;
  d.msg_grid = best_grid;
  d.msg_shape = best_shape;
  d.sparse_div = sparse_div;
  HIPCHK(s, hipGetLastError());
  return ABM_OK;
}

int check_dev_flags(abm_sim* s) {
  int32_t f = 0;
  HIPCHK(s, hipMemcpyAsync(&f, s->d.flags, sizeof f, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  if (f & FLAG_CAPACITY)
    return s->fail(ABM_E_CAPACITY, "a day's contact graph exceeded the edge room (%lld edges)",
                   (long long)s->z.ecap);
  if (f & FLAG_RECV_OVERFLOW) return s->fail(ABM_E_CAPACITY, "received-contact counter overflow");
  return ABM_OK;
}

}  // namespace

#include "soft_driver.inc"

extern "C" {

int abm_workspace_size(const abm_params* p, const abm_population* pop, size_t* bytes) {
  if (!bytes) return ABM_E_ARG;
  Sizes z;
  std::string why;
  const int rc = validate(p, pop, z, why);
  if (rc) return rc;
  Offsets o;
  layout(z, *p, o, *bytes);
  return ABM_OK;
}

int abm_create(const abm_params* p, const abm_population* pop, void* d_workspace, size_t ws_bytes,
               void* hip_stream, abm_sim** out) {
  if (!out) return ABM_E_ARG;
  *out = nullptr;
  abm_sim* s = new abm_sim();
  *out = s;
  std::string why;
  int rc = validate(p, pop, s->z, why);
  if (rc) return s->fail(rc, "%s", why.c_str());
  s->p = *p;
  const Sizes& z = s->z;
  size_t need = 0;
  layout(z, *p, s->o, need);
  if (!d_workspace || ws_bytes < need)
    return s->fail(ABM_E_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  s->ws = (char*)d_workspace;
  s->stream = (hipStream_t)hip_stream;
  const Offsets& o = s->o;
  char* ws = s->ws;
  Dev& d = s->d;
  d.N = (int32_t)z.N;
  d.R = (int32_t)z.R;
  d.ntiles = (int32_t)z.ntiles;
  d.T = (int32_t)z.T;
  d.ecap = z.ecap;
  d.nscan = (int32_t)z.nscan;
  d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
  d.key1 = (uint32_t)(p->seed >> 32);
  d.e_days = p->e_days;
  d.i_days = p->i_days;
  d.qdays = p->quarantine_days;
  d.test_delay = p->test_delay;
  d.dose_lag = p->dose_lag;
  d.vacc_on = p->vacc_rate > 0 ? 1 : 0;
  d.strategy = p->strategy;
  d.mode = p->mode;
  d.course_on = p->disease_model == ABM_DISEASE_COURSE ? 1 : 0;
  for (int k = 0; k < ABM_N_DUR; ++k) d.dur_shift[k] = p->dur_shift[k];
  d.w_h = p->w_household;
  d.w_o = p->w_occupation;
  d.w_r = p->w_random;
  d.dt = p->dt;
  d.test_rate = p->test_rate;
  d.sens = p->test_sensitivity;
  d.dropout = p->quarantine_dropout;
  d.eff1 = p->eff1;
  d.eff2 = p->eff2;
  d.gtau = p->gumbel_tau;
  d.kappa = p->kappa;
  d.vacc_trigger = p->vacc_trigger;
  for (int a = 0; a < ABM_N_AGE; ++a) {
    d.p_death[a] = p->p_death[a];
    d.cprob[0][a] = p->p_asym[a];
    d.cprob[1][a] = p->p_severe[a];
    d.cprob[2][a] = p->p_hosp[a];
    d.cprob[3][a] = p->p_icu[a];
    d.cprob[4][a] = p->p_die[a];
    d.vrank[0][a] = (int8_t)priority_class(p->strategy, 1, a);
    d.vrank[1][a] = (int8_t)priority_class(p->strategy, 2, a);
  }
  d.rep = (const RepInfo*)(ws + o.rep);
  d.tiles = (const int4*)(ws + o.tiles);
  d.srec = (const StaticRec*)(ws + o.srec);
  d.age = (const uint8_t*)(ws + o.age);
  d.hhn = (const uint8_t*)(ws + o.hhn);
  d.wp_members = (const int32_t*)(ws + o.wpm);
  d.atab = (const float*)(ws + o.atab);
  d.ptab = (const uint32_t*)(ws + o.ptab);
  d.dtab = (const uint32_t*)(ws + o.dtab);
  d.state = (AgentState*)(ws + o.state);
  d.code = (uint8_t*)(ws + o.code);
  d.imask = (uint32_t*)(ws + o.imask);
  d.cmask = (uint32_t*)(ws + o.cmask);
  d.scmask = (unsigned long long*)(ws + o.scmask);
  d.nsc = (int32_t)((z.N + 16383) / 16384);
  d.lambda = (float*)(ws + o.lambda);
  d.own = (uint16_t*)(ws + o.own);
  d.recv = (uint32_t*)(ws + o.recv);
  d.ring_n = (int32_t)ring_slots(z, *p);
  if (d.ring_n == 1) d.row_ptr = (int32_t*)(ws + o.row_ptr);
  d.cur_occ = (int32_t*)(ws + o.cur_occ);
  d.cur_rand = (int32_t*)(ws + o.cur_rand);
  if (d.ring_n == 1) d.col = (int32_t*)(ws + o.col);
  d.scan_part = (int64_t*)(ws + o.scan_part);
  d.vhist = (int32_t*)(ws + o.vhist);
  d.vplan = (int32_t*)(ws + o.vplan);
  d.vtile_base = (int32_t*)(ws + o.vtile);
  d.latch = (uint8_t*)(ws + o.latch);
  d.vseg = (int32_t)z.vseg;
  d.vpart = z.vseg ? (int32_t*)(ws + o.vpart) : nullptr;
  d.vsegbase = z.vseg ? (int32_t*)(ws + o.vsegbase) : nullptr;
  d.tile_counts = (uint32_t*)(ws + o.tile_counts);
  d.fin_part = (unsigned long long*)(ws + o.fin_part);
  d.fseg = (int32_t)z.fseg;
  d.fin_one = (int32_t)z.fin_one;
  d.prev_counts = (long long*)(ws + o.prev_counts);
  d.traj = (long long*)(ws + o.traj);
  d.day = (int32_t*)(ws + o.day);
  d.fin_done = d.day + 1;
  d.rmask = (uint32_t*)(ws + o.rmask);
  d.ninf = (int32_t*)(ws + o.ninf);
  d.work = (int32_t*)(ws + o.work);
  d.nwork = (int32_t*)(ws + o.nwork);
  d.work_cap = (int32_t)front_cap(z);
  d.sparse_div = (p->flags & ABM_FLAG_DENSE_MESSAGE) ? 0
                 : (z.N >= FRONT_MIN_N || (p->flags & ABM_FLAG_FRONTIER_ANY_SIZE)) ? SPARSE_DIV : 0;
  d.test_dmin = p->test_delay;
  d.test_dmax = p->test_delay_max;
  d.immune_asym = p->vacc_immunity == ABM_IMMUNITY_ASYMPTOMATIC ? 1 : 0;
  d.straight = (p->flags & ABM_FLAG_STRAIGHT_THROUGH) ? 1 : 0;
  d.den_on = p->app_adoption > 0.f ? 1 : 0;
  d.den_window = p->den_window;
  d.den_adoption = p->app_adoption;
  d.den_compliance = p->den_compliance;
  if (d.ring_n > 1) {
    d.ring_rp = (int32_t*)(ws + o.ring_rp);
    d.ring_col = (int32_t*)(ws + o.ring_col);
    d.ring_rstride = ring_rstride(z);
    d.ring_cstride = ring_cstride(z);
    d.row_ptr = d.ring_rp;                 // slot 0: day 0's graph
    d.col = d.ring_col;
  }
  if (d.den_on) d.den_mask = (uint32_t*)(ws + o.den_mask);
  d.flags = (int32_t*)(ws + o.flags);
  if (p->mode == ABM_SOFT) {
    d.s = (float*)(ws + o.s);
    d.ehist = (float*)(ws + o.ehist);
    d.inf = (float*)(ws + o.inf);
    d.sigma = (float*)(ws + o.sigma);
    d.soft_inc = (float*)(ws + o.soft_inc);
    d.seg_sigma = (float*)(ws + o.seg_sigma);
    d.seg_y = (float*)(ws + o.seg_y);
    d.seg_s = (float*)(ws + o.seg_s);
    d.ckpt = (float*)(ws + o.ckpt);
    d.s_bar = (float*)(ws + o.s_bar);
    d.ibar = (float*)(ws + o.ibar);
    d.vtmp = (float*)(ws + o.vtmp);
    d.lam_bar = (float*)(ws + o.lam_bar);
    d.gtheta = (float*)(ws + o.gtheta);
    d.gpart = (float*)(ws + o.gpart);
    d.dL = (const float*)(ws + o.dL);
    d.seg = (int32_t)z.seg;
  }
  d.msg_chunk = 4096;
  d.msg_grid = d.ntiles;
  d.msg_shape = 0;
  d.pb_on = (int32_t)z.pb_on;
  if (z.pb_on) {
    d.pb_lb = (int32_t)z.lb;
    d.pb_nlv = (int32_t)z.nlv;
    d.pb_nb1 = (int32_t)z.nb1;
    d.pb_nbatch = (int32_t)z.nbatch;
    d.pb_bpw = (int32_t)z.bpw;
    d.pb_ngrid = (int32_t)z.ngrid;
    d.pb_bcap = (int32_t)z.bcap;
    d.pb_s1_nparts = (int32_t)z.s1_nparts;
    d.pb_maxch = (int32_t)z.maxch;
    d.pb_nleaf = (int32_t)z.nleaf;
    d.pb_rper = (int32_t)z.rper;
    d.pb_asm_cap = (int32_t)z.asm_cap;
    d.pb_s1_cap = (int32_t)z.s1_cap;
    d.pb_ccap = z.ccap;
    d.pb_hist1 = (int32_t*)(ws + o.pb_hist1);
    d.pb_own = (uint32_t*)(ws + o.pb_own);
    d.pb_tbase = (int2*)(ws + o.pb_tbase);
    d.pb_part = (int64_t*)(ws + o.pb_part);
    d.pb_bstart = (int32_t*)(ws + o.pb_bstart);
    d.pb_bchunk = (int32_t*)(ws + o.pb_bchunk);
    d.pb_nchunks = (int32_t*)(ws + o.pb_nchunks);
    d.pb_chunks = (int4*)(ws + o.pb_chunks);
    d.pb_hist2 = (int32_t*)(ws + o.pb_hist2);
    d.pb_leaf = (int32_t*)(ws + o.pb_leaf);
    d.pb_b1h = (uint16_t*)(ws + o.pb_b1h);
    d.pb_b1w = (uint32_t*)(ws + o.pb_b1w);
    d.pb_buf2 = (uint2*)(ws + o.pb_buf2);
    d.pb_sh = (int32_t)(z.lb - 8);
    d.pb_tdeg = (int32_t*)(ws + o.pb_tdeg);
    d.pb_tstart = (int32_t*)(ws + o.pb_tstart);
    d.pb_tpart = (int64_t*)(ws + o.pb_tpart);
    d.pb_ntgrp = (int32_t)((z.nlv + 1023) / 1024);
  }
  name_kernels(s);

  // host copies of the static data
  const int64_t N = z.N;
  const int R = (int)z.R;
  std::vector<StaticRec> srec(N);
  std::vector<uint8_t> hhn(N);
  for (int h = 0; h < pop->n_households; ++h)
    for (int64_t i = pop->hh_start[h]; i < pop->hh_start[h + 1]; ++i) {
      srec[i].hh_lo = pop->hh_start[h];
      srec[i].hh_n = (uint8_t)(pop->hh_start[h + 1] - pop->hh_start[h]);
      hhn[i] = srec[i].hh_n;
    }
  std::vector<int32_t> agent_rep(N);
  for (int r = 0; r < R; ++r)
    for (int64_t i = pop->agent_offset[r]; i < pop->agent_offset[r + 1]; ++i) agent_rep[i] = r;
  for (int64_t i = 0; i < N; ++i) {
    srec[i].age = pop->age[i];
    srec[i].occ = pop->occupation[i];
    srec[i].pad = 0;
    srec[i].wp_lo = 0;
    srec[i].wp_pos = 0;
    srec[i].wp_n = 0;
  }
  std::vector<uint8_t> seen(N, 0);
  for (int w = 0; w < pop->n_workplaces; ++w) {
    const int32_t lo = pop->wp_start[w], hi = pop->wp_start[w + 1];
    const int r0 = agent_rep[pop->wp_members[lo]];
    for (int32_t q = lo; q < hi; ++q) {
      const int32_t a = pop->wp_members[q];
      if (seen[a]) return s->fail(ABM_E_ARG, "agent %d belongs to two workplaces", a);
      if (agent_rep[a] != r0) return s->fail(ABM_E_ARG, "workplace %d crosses replicates", w);
      seen[a] = 1;
      srec[a].wp_lo = lo;
      srec[a].wp_pos = (uint16_t)(q - lo);
      srec[a].wp_n = (uint16_t)(hi - lo);
    }
  }
  s->reps.resize(R);
  std::vector<int4> tiles;
  tiles.reserve(z.ntiles);
  const float kappa = p->kappa;
  for (int r = 0; r < R; ++r) {
    RepInfo& ri = s->reps[r];
    memset(&ri, 0, sizeof ri);
    ri.start = (int32_t)pop->agent_offset[r];
    ri.n = (int32_t)(pop->agent_offset[r + 1] - pop->agent_offset[r]);
    ri.stream = pop->stream ? pop->stream[r] : (uint32_t)r;
    ri.delay = pop->dose2_delay[r];
    ri.cap = (int64_t)std::floor(p->vacc_rate * (double)ri.n);
    ri.tile0 = (int32_t)tiles.size();
    for (int32_t a = ri.start; a < ri.start + ri.n; a += TILE) {
      const int32_t b = std::min(a + TILE, ri.start + ri.n);
      tiles.push_back(make_int4(r, a, b, (int)tiles.size()));
    }
    ri.ntiles = (int32_t)tiles.size() - ri.tile0;
    ri.R = pop->R[r];
    const float rk = ri.R * kappa;
    ri.rk = rk;
    for (int a = 0; a < ABM_N_AGE; ++a) {
      ri.S[a] = pop->susceptibility[r * ABM_N_AGE + a];
      ri.coef[a] = rk * ri.S[a];
    }
  }
  float atab[ATAB];
  if (p->disease_model == ABM_DISEASE_COURSE)
    build_atab_course(*p, atab);
  else
    build_atab(*p, atab);
  std::vector<uint32_t> dtab(ABM_N_DUR * 64);
  for (int k = 0; k < ABM_N_DUR; ++k) build_poisson(p->dur_extra[k], &dtab[k * 64]);
  std::vector<uint32_t> ptab(NPT * 64);
  for (int k = 0; k < ABM_N_OCC; ++k) build_poisson(p->mu_occupation[k] / 2.0, &ptab[k * 64]);
  for (int a = 0; a < ABM_N_AGE; ++a) build_poisson(p->mu_random[a] / 2.0, &ptab[(PT_AGE0 + a) * 64]);

  hipStream_t st = s->stream;
  HIPCHK(s, hipMemcpyAsync(ws + o.rep, s->reps.data(), R * sizeof(RepInfo), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.srec, srec.data(), N * sizeof(StaticRec), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.age, pop->age, N, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.hhn, hhn.data(), N, hipMemcpyHostToDevice, st));
  if (z.M > 0)
    HIPCHK(s, hipMemcpyAsync(ws + o.wpm, pop->wp_members, z.M * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.atab, atab, sizeof atab, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.ptab, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(ws + o.dtab, dtab.data(), dtab.size() * 4, hipMemcpyHostToDevice, st));
  if (z.nseeds > 0)
    HIPCHK(s, hipMemcpyAsync(ws + o.seeds, pop->initial_infected, z.nseeds * 4, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemsetAsync(ws + o.latch, 0, R, st));
  HIPCHK(s, hipMemsetAsync(ws + o.day, 0, 8, st));
  HIPCHK(s, hipMemsetAsync(ws + o.ninf, 0, 4, st));
  if (d.den_on) {                          // no graphs before day 0: empty rows
    HIPCHK(s, hipMemsetAsync(ws + o.ring_rp, 0, (size_t)p->den_window * d.ring_rstride * 4, st));
    HIPCHK(s, hipMemsetAsync(ws + o.den_mask, 0, ((N + 31) / 32 + 1) * 4, st));
  }
  HIPCHK(s, hipMemsetAsync(ws + o.flags, 0, 4, st));
  HIPCHK(s, hipMemsetAsync(ws + o.vplan, 0, 8 * R, st));
  HIPCHK(s, hipMemsetAsync(ws + o.traj, 0, z.T * z.R * ABM_NC * 8, st));
  launch_init_state(d, (const int32_t*)(ws + o.seeds), z.nseeds, st);
  launch_recount(d, st);
  if (p->mode == ABM_SOFT) {
    rc = soft_create(s);
    if (rc) return rc;
  }
  HIPCHK(s, prepare_build(d));
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipStreamSynchronize(st));
  if ((p->flags & ABM_FLAG_AUTOTUNE) && p->mode == ABM_HARD) {
    rc = autotune(s);
    if (rc) return rc;
  }
  const bool use_graph = !(p->flags & (ABM_FLAG_PROFILE | ABM_FLAG_NO_GRAPH)) && p->mode == ABM_HARD;
  if (use_graph) {
    HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    const int ng = d.den_on ? d.den_window : 1;
    s->graphs.assign(ng, nullptr);
    s->execs.assign(ng, nullptr);
    for (int g = 0; g < ng; ++g) {
      HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
      enqueue_day(s, g, s->cap_stream, nullptr);
      HIPCHK(s, hipStreamEndCapture(s->cap_stream, &s->graphs[g]));
      HIPCHK(s, hipGraphInstantiate(&s->execs[g], s->graphs[g], nullptr, nullptr, 0));
    }
  }
  return ABM_OK;
}

int abm_step(abm_sim* s, int32_t n_days) {
  if (!s) return ABM_E_ARG;
  if (s->err) return s->err;
  if (n_days < 0) return s->fail(ABM_E_ARG, "n_days < 0");
  if (s->p.mode != ABM_HARD) return s->fail(ABM_E_STATE, "abm_step is for hard mode; use abm_run");
  if ((int64_t)s->host_day + n_days > s->z.T)
    return s->fail(ABM_E_STATE, "stepping past n_steps (%d)", (int)s->z.T);
  const bool timed = (s->p.flags & ABM_FLAG_PROFILE) != 0;
  for (int k = 0; k < n_days; ++k) {
    if (!s->execs.empty()) {
      HIPCHK(s, hipGraphLaunch(s->execs[s->host_day % s->execs.size()], s->stream));
    } else if (timed) {
      if (s->prof_used == s->prof_sets.size()) {
        std::vector<hipEvent_t> ev(s->nk + 1);
        for (auto& e : ev) HIPCHK(s, hipEventCreate(&e));
        s->prof_sets.push_back(ev);
      }
      const std::vector<hipEvent_t>* ev = &s->prof_sets[s->prof_used];
      ++s->prof_used;
      enqueue_day(s, s->host_day, s->stream, ev);
      HIPCHK(s, hipGetLastError());
    } else {
      enqueue_day(s, s->host_day, s->stream, nullptr);
      HIPCHK(s, hipGetLastError());
    }
    ++s->host_day;
  }
  return ABM_OK;
}

int abm_run(abm_sim* s, int32_t n_days, int64_t* h_counts, float* h_soft_incidence) {
  if (!s) return ABM_E_ARG;
  if (s->err) return s->err;
  if (s->p.mode == ABM_SOFT) return soft_run(s, n_days, h_soft_incidence);
  const int32_t t0 = s->host_day;
  int rc = abm_step(s, n_days);
  if (rc) return rc;
  rc = check_dev_flags(s);
  if (rc) return rc;
  if (h_counts && n_days > 0) {
    const size_t row = (size_t)s->z.R * ABM_NC;
    HIPCHK(s, hipMemcpyAsync(h_counts, s->d.traj + (size_t)t0 * row, n_days * row * 8,
                             hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
  }
  return ABM_OK;
}

int abm_get(abm_sim* s, int32_t what, void* h_dst, size_t h_bytes) {
  if (!s || !h_dst) return ABM_E_ARG;
  if (s->err) return s->err;
  const int rc = check_dev_flags(s);
  if (rc) return rc;
  const int64_t N = s->z.N;
  const void* src = nullptr;
  size_t n = 0;
  int32_t E = 0;
  // the graph of the last day built (day 0's before the first step)
  const Dev last = day_dev(s, std::max(0, s->host_day - 1));
  if (what == ABM_GET_COL || what == ABM_GET_W) {
    HIPCHK(s, hipMemcpy(&E, last.row_ptr + N, 4, hipMemcpyDeviceToHost));
  }
  switch (what) {
    case ABM_GET_STATE: src = s->d.state; n = N * sizeof(AgentState); break;
    case ABM_GET_LAMBDA: src = s->d.lambda; n = N * 4; break;
    case ABM_GET_CODE: src = s->d.code; n = N; break;
    case ABM_GET_ROWPTR: src = last.row_ptr; n = (N + 1) * 4; break;
    case ABM_GET_COL: src = last.col; n = (size_t)E * 4; break;
    case ABM_GET_W: src = last.col; n = (size_t)E * 4; break;   // decoded below
    case ABM_GET_ATAB: src = s->d.atab; n = ATAB * 4; break;
    case ABM_GET_POISSON: src = s->d.ptab; n = NPT * 64 * 4; break;
    case ABM_GET_LATCH: src = s->d.latch; n = s->z.R; break;
    case ABM_GET_SOFT_S:
      if (s->p.mode != ABM_SOFT) return s->fail(ABM_E_STATE, "not a soft-mode simulation");
      src = s->d.s; n = N * 4; break;
    case ABM_GET_DAY:
      if (h_bytes < 4) return s->fail(ABM_E_ARG, "buffer too small");
      *(int32_t*)h_dst = s->host_day;
      return ABM_OK;
    case ABM_GET_TUNING: {
      if (h_bytes < 12) return s->fail(ABM_E_ARG, "buffer too small");
      int32_t* v = (int32_t*)h_dst;
      v[0] = s->d.msg_chunk;
      v[1] = s->d.msg_grid;
      v[2] = s->d.msg_shape;
      return ABM_OK;
    }
    case ABM_GET_COEF: {
      if (h_bytes < (size_t)s->z.R * ABM_N_AGE * 4) return s->fail(ABM_E_ARG, "buffer too small");
      float* f = (float*)h_dst;
      for (int r = 0; r < s->z.R; ++r)
        for (int a = 0; a < ABM_N_AGE; ++a) f[r * ABM_N_AGE + a] = s->reps[r].coef[a];
      return ABM_OK;
    }
    default: return s->fail(ABM_E_ARG, "unknown abm_get item %d", what);
  }
  if (h_bytes < n) return s->fail(ABM_E_ARG, "buffer of %zu bytes, %zu needed", h_bytes, n);
  if (n) {
    HIPCHK(s, hipMemcpyAsync(h_dst, src, n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
  }
  // column words carry the contact network in their top two bits: split into the
  // source agent (ABM_GET_COL) or the network's weight (ABM_GET_W)
  if (what == ABM_GET_COL) {
    uint32_t* c = (uint32_t*)h_dst;
    for (int32_t e = 0; e < E; ++e) c[e] &= 0x3FFFFFFFu;
  } else if (what == ABM_GET_W) {
    const float wt[4] = {s->p.w_household, s->p.w_occupation, s->p.w_random, s->p.w_random};
    char* b = (char*)h_dst;
    for (int32_t e = 0; e < E; ++e) {
      uint32_t c;
      std::memcpy(&c, b + 4 * (size_t)e, 4);
      std::memcpy(b + 4 * (size_t)e, &wt[c >> 30], 4);
    }
  }
  return ABM_OK;
}

int abm_set_state(abm_sim* s, int32_t day, const uint8_t* h_latch, const abm_agent_state* h_state,
                  size_t n_agents) {
  if (!s || !h_state || !h_latch) return ABM_E_ARG;
  if (s->err) return s->err;
  if (s->p.mode != ABM_HARD) return s->fail(ABM_E_STATE, "abm_set_state is for hard mode");
  if ((int64_t)n_agents != s->z.N) return s->fail(ABM_E_ARG, "state of %zu agents, %lld expected",
                                                 n_agents, (long long)s->z.N);
  if (day < 0 || day > s->z.T) return s->fail(ABM_E_ARG, "day out of range");
  HIPCHK(s, hipMemcpyAsync(s->d.state, h_state, n_agents * sizeof(AgentState), hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipMemcpyAsync(s->d.latch, h_latch, s->z.R, hipMemcpyHostToDevice, s->stream));
  if (s->d.den_on) {
    // the notification ring holds the graphs of the den_window days before `day`
    HIPCHK(s, hipMemsetAsync(s->ws + s->o.ring_rp, 0, (size_t)s->d.den_window * s->d.ring_rstride * 4, s->stream));
    HIPCHK(s, hipMemsetAsync(s->ws + s->o.den_mask, 0, ((s->z.N + 31) / 32 + 1) * 4, s->stream));
    for (int32_t dd = std::max(0, day - s->d.den_window); dd < day; ++dd) {
      const Dev dv = day_dev(s, dd);
      launch_set_day(dv, dd, s->stream);
      for (int b = 0; b < build_steps(dv); ++b) launch_build_step(dv, b, s->stream);
    }
  }
  launch_set_day(s->d, day, s->stream);
  launch_recount(s->d, s->stream);
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->host_day = day;
  return ABM_OK;
}

int abm_sync(abm_sim* s) {
  if (!s) return ABM_E_ARG;
  if (s->err) return s->err;
  return check_dev_flags(s);
}

void abm_destroy(abm_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto e : s->execs)
    if (e) (void)hipGraphExecDestroy(e);
  for (auto g : s->graphs)
    if (g) (void)hipGraphDestroy(g);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  for (auto& ev : s->prof_sets)
    for (auto e : ev) (void)hipEventDestroy(e);
  delete s;
}

const char* abm_error_string(int code) {
  switch (code) {
    case ABM_OK: return "ok";
    case ABM_E_ARG: return "invalid argument";
    case ABM_E_ABI: return "ABI mismatch";
    case ABM_E_WORKSPACE: return "workspace too small";
    case ABM_E_CAPACITY: return "edge capacity exceeded";
    case ABM_E_HIP: return "HIP runtime error";
    case ABM_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

const char* abm_last_error(const abm_sim* s) { return s ? s->msg.c_str() : "null simulation"; }

int abm_profile_kernels(const abm_sim* s) { return s ? s->nk : 0; }
const char* abm_profile_name(const abm_sim* s, int32_t k) {
  return (s && k >= 0 && k < s->nk) ? s->names[k].c_str() : "";
}
int abm_profile_get(abm_sim* s, double* h_ms, int64_t* h_launches) {
  if (!s) return ABM_E_ARG;
  if (s->err) return s->err;
  const int rc = drain_profile(s);
  if (rc) return rc;
  for (int k = 0; k < s->nk; ++k) {
    if (h_ms) h_ms[k] = s->ms[k];
    if (h_launches) h_launches[k] = s->launches[k];
  }
  return ABM_OK;
}
int abm_profile_reset(abm_sim* s) {
  if (!s) return ABM_E_ARG;
  if (s->err) return s->err;
  const int rc = drain_profile(s);
  if (rc) return rc;
  for (int k = 0; k < s->nk; ++k) {
    s->ms[k] = 0;
    s->launches[k] = 0;
  }
  return ABM_OK;
}

int abm_philox(uint64_t seed, const uint32_t* d_ctr, int64_t n, uint32_t* d_out, void* hip_stream) {
  if (n < 0 || (n > 0 && (!d_ctr || !d_out))) return ABM_E_ARG;
  launch_philox(seed, d_ctr, n, d_out, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? ABM_OK : ABM_E_HIP;
}

}  // extern "C"
