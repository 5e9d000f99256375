// Per-day agent kernels: interventions before transmission, the edge-message force of
// infection (eq. 1), the fused infection / progression / testing / vaccination step
// (eq. 2; sections 3-5), and the end-of-day bookkeeping.
#include <algorithm>

#include "abm_internal.h"

namespace abm {

// ---- small block helpers (TILE = 256 threads = 4 waves of 64) -----------------------
__device__ __forceinline__ uint32_t wave_count(bool p) {
  return (uint32_t)__popcll(__ballot(p));
}

// Sum `nv` per-thread boolean counters over the workgroup and add them to dst[slot[k]].
template <int NV>
__device__ __forceinline__ void block_count_add(const bool (&v)[NV], const int (&slot)[NV],
                                                unsigned long long* dst) {
  __shared__ uint32_t part[TILE / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const uint32_t c = wave_count(v[k]);
    if (lane == 0) part[wv][k] = c;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    uint32_t s = 0;
    for (int q = 0; q < TILE / 64; ++q) s += part[q][threadIdx.x];
    if (s) atomicAdd(&dst[slot[threadIdx.x]], (unsigned long long)s);
  }
}

// Sum per-thread boolean counters over the workgroup and store them in this tile's row
// of the per-tile count table (one writer per slot per day: no atomics).
template <int NV>
__device__ __forceinline__ void block_count_store(const bool (&v)[NV], const int (&slot)[NV],
                                                  uint32_t* row) {
  __shared__ uint32_t part[TILE / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const uint32_t c = wave_count(v[k]);
    if (lane == 0) part[wv][k] = c;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    uint32_t s = 0;
    for (int q = 0; q < TILE / 64; ++q) s += part[q][threadIdx.x];
    row[slot[threadIdx.x]] = s;
  }
}

__device__ __forceinline__ int vacc_bucket(const Dev& d, const AgentState& a, int t, int age,
                                           int delay) {
  if (a.stage == ABM_STAGE_M) return NBUCKET;
  if (a.vacc == 0) return d.vrank[0][age];
  if (a.vacc == 1 && t >= (int)a.d1 + delay) return d.vrank[1][age];
  return NBUCKET;
}

// ---- testing turnaround and digital exposure notification (section 4) ----------------
// App access: lane 0 of purpose APP on day 0, below the adoption share.
__device__ __forceinline__ bool app_user(const Dev& d, uint32_t loc, uint32_t stream) {
  return u01(philox(loc, 0u, stream, P_APP << 24, d.key0, d.key1).x) < d.den_adoption;
}
// Days from a test to its result: uniform over test_dmin..test_dmax from lane 1 of
// AGENT2 on the test day, k = floor(x n / 2^32).
__device__ __forceinline__ int result_delay(const Dev& d, uint32_t loc, uint32_t stream, int test_day) {
  const uint32_t n = (uint32_t)(d.test_dmax - d.test_dmin + 1);
  if (n <= 1u) return d.test_dmin;
  const uint32_t x = philox(loc, (uint32_t)test_day, stream, P_AGENT2 << 24, d.key0, d.key1).y;
  return d.test_dmin + (int)(((uint64_t)x * n) >> 32);
}

// ---- eleven-stage course (section 3, "Agent State Definition", "Disease Progression") --
// An infection on day t draws the whole path from lanes 0..3 of the course's block 0
// (asymptomatic with p_asym[a], else severe with p_severe[a], else mild; a severe
// course is hospitalised with p_hosp[a]; a hospitalised one reaches intensive care with
// p_icu[a]).  Every stage's duration is shift + Poisson(extra) days, from lane 0 of block
// 1 on the day the stage starts; whether intensive care ends in death is lane 1 of
// that block on the day it starts (p_die[a]).
__device__ __forceinline__ int course_days(const Dev& d, int k, uint32_t x) {
  return d.dur_shift[k] + poisson_k(d.dtab + k * 64, x);
}

// (`protected_`: a vaccine-protected agent under asymptomatic immunity takes the
// asymptomatic course whatever its draw)
__device__ __forceinline__ void course_infect(const Dev& d, AgentState& a, uint32_t loc, int t,
                                              uint32_t stream, int age, bool protected_ = false) {
  const uint4 b0 = philox(loc, (uint32_t)t, stream, P_COURSE << 24, d.key0, d.key1);
  const uint4 b1 = philox(loc, (uint32_t)t, stream, (P_COURSE << 24) | 1u, d.key0, d.key1);
  const bool asym = protected_ || u01(b0.x) < d.cprob[0][age];
  const bool severe = !asym && u01(b0.y) < d.cprob[1][age];
  const bool hosp = severe && u01(b0.z) < d.cprob[2][age];
  const bool icu = hosp && u01(b0.w) < d.cprob[3][age];
  a.course = (uint8_t)((asym ? 0 : (severe ? 2 : 1)) | (hosp ? 4 : 0) | (icu ? 8 : 0));
  a.stage = (uint8_t)(asym ? ABM_STAGE_ASYM : (severe ? ABM_STAGE_PRE_SEVERE : ABM_STAGE_PRE_MILD));
  a.t_next = (int16_t)(t + course_days(d, asym ? ABM_DUR_ASYM : ABM_DUR_PRE, b1.x));
}

// The transition of an agent whose current stage ends on day t.
__device__ __forceinline__ void course_step(const Dev& d, AgentState& a, uint32_t loc, int t,
                                            uint32_t stream, int age) {
  const int c = a.course;
  int next = ABM_STAGE_R, k = -1;
  switch (a.stage) {
    case ABM_STAGE_PRE_MILD: next = ABM_STAGE_MILD; k = ABM_DUR_MILD; break;
    case ABM_STAGE_PRE_SEVERE:
      next = ABM_STAGE_SEVERE;
      k = (c & 4) ? ABM_DUR_SEV_HOSP : ABM_DUR_SEV_R;
      break;
    case ABM_STAGE_SEVERE:
      if (c & 4) {
        next = ABM_STAGE_HOSP;
        k = (c & 8) ? ABM_DUR_HOSP_ICU : ABM_DUR_HOSP_R;
      }
      break;
    case ABM_STAGE_HOSP:
      if (c & 8) next = ABM_STAGE_ICU;
      break;
    case ABM_STAGE_ICU: next = (c & 16) ? ABM_STAGE_M : ABM_STAGE_R; break;
    default: break;                               // asymptomatic and mild recover
  }
  if (k >= 0 || next == ABM_STAGE_ICU) {
    const uint4 b1 = philox(loc, (uint32_t)t, stream, (P_COURSE << 24) | 1u, d.key0, d.key1);
    if (next == ABM_STAGE_ICU) {
      const bool die = u01(b1.y) < d.cprob[4][age];
      a.course = (uint8_t)(c | (die ? 16 : 0));
      k = die ? ABM_DUR_ICU_DIE : ABM_DUR_ICU_R;
    }
    a.t_next = (int16_t)(t + course_days(d, k, b1.x));
  } else {
    a.t_next = (int16_t)ABM_NEVER;
  }
  a.stage = (uint8_t)next;
}

// Count groups: E counts the infected without symptoms, I the symptomatic outside hospital.
__device__ __forceinline__ bool stage_e(int st) {
  return st == ABM_STAGE_E || st == ABM_STAGE_ASYM || st == ABM_STAGE_PRE_MILD || st == ABM_STAGE_PRE_SEVERE;
}
__device__ __forceinline__ bool stage_i(int st) {
  return st == ABM_STAGE_I || st == ABM_STAGE_MILD || st == ABM_STAGE_SEVERE;
}

// ---- pre: results due -> quarantine, dropout, infectiousness codes, vaccine classes --
__global__ __launch_bounds__(TILE) void k_pre(Dev d) {
  __shared__ int hist[NBUCKET + 1];
  if (threadIdx.x <= NBUCKET) hist[threadIdx.x] = 0;
  __syncthreads();
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const bool live = i < tl.z;
  const int t = *d.day;
  bool pos_due = false;
  if (live) {
    const RepInfo& ri = d.rep[tl.x];
    AgentState a = d.state[i];
    const AgentState a0 = a;
    const uint32_t loc = (uint32_t)(i - ri.start);
    if ((a.flags & 1) && t == (int)a.test_day + result_delay(d, loc, ri.stream, a.test_day)) {
      if (a.flags & 2) {
        pos_due = true;
        if (d.qdays > 0) a.q_until = (int16_t)(t + d.qdays);
      }
      a.flags = (uint8_t)(a.flags & ~3);
    }
    // a positive app user notifies every contact of the last den_window days (its rows
    // of those days' graphs; the graph is symmetric); the contacts check app access and
    // quarantine themselves in the fused step
    if (d.den_on && pos_due && app_user(d, loc, ri.stream)) {
      for (int k = 1; k <= d.den_window && t - k >= 0; ++k) {
        const int slot = (t - k) % d.den_window;
        const int32_t* rp = d.ring_rp + (size_t)slot * d.ring_rstride;
        const int32_t* col = d.ring_col + (size_t)slot * d.ring_cstride;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
          const uint32_t j = (uint32_t)col[e] & COL_AGENT;
          atomicOr(&d.den_mask[j >> 5], 1u << (j & 31));
        }
      }
    }
    if (d.dropout > 0.f && t < (int)a.q_until) {
      const uint4 b = philox((uint32_t)(i - ri.start), (uint32_t)t, ri.stream, P_AGENT2 << 24,
                             d.key0, d.key1);
      if (u01(b.x) < d.dropout) a.q_until = (int16_t)t;
    }
    uint8_t c = 0;
    if (d.course_on) {
      // 16 * class + days since exposure: asymptomatic 1, presymptomatic 2, symptomatic 3
      const int st = a.stage, tau = t - (int)a.t_exp;
      const int cls = st == ABM_STAGE_ASYM ? 1
                      : (st == ABM_STAGE_PRE_MILD || st == ABM_STAGE_PRE_SEVERE) ? 2
                      : (st == ABM_STAGE_MILD || st == ABM_STAGE_SEVERE) ? 3 : 0;
      if (cls && tau >= 1 && tau <= 15 && t >= (int)a.q_until) c = (uint8_t)(16 * cls + tau);
    } else if ((a.stage == ABM_STAGE_E || a.stage == ABM_STAGE_I) && t >= (int)a.q_until) {
      c = (uint8_t)(t - (int)a.t_exp);
    }
    d.code[i] = c;
    if (a.flags != a0.flags || a.q_until != a0.q_until) d.state[i] = a;
    if (d.vacc_on) atomicAdd(&hist[vacc_bucket(d, a, t, d.age[i], ri.delay)], 1);
  }
  const bool v[1] = {pos_due};
  const int sl[1] = {ABM_C_POS};
  block_count_store<1>(v, sl, d.tile_counts + (size_t)blockIdx.x * TILE_NC);
  if (d.vacc_on) {
    __syncthreads();
    if (threadIdx.x < NBUCKET) d.vhist[(size_t)blockIdx.x * NBUCKET + threadIdx.x] = hist[threadIdx.x];
  }
  // the frontier counters start afresh today (stored last: a store before the tile's
  // loads would keep the compiler from loading the tile record through the scalar cache)
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) *d.ninf = 0;
    for (int q = threadIdx.x; q < FRONT_NB; q += TILE) d.nwork[q] = 0;
  }
}

// ---- infectious bit masks ---------------------------------------------------------
// Fine: bit i = agent i infectious today (one 32-bit word per 32 agents, 1/8 byte per
// agent).  Coarse: bit g = some agent of the group [8g, 8g+8) infectious (1/64 byte per
// agent, small enough to stay in L2).  The message kernel tests the coarse bit, then the
// fine bit, before it reads an edge's weight and the source's code byte.
// One lane per fine word (32 agents); a workgroup of MASK_T lanes covers one
// super-coarse word (64 coarse words of 256 agents).
constexpr int MASK_T = 512;
__global__ __launch_bounds__(MASK_T) void k_mask(Dev d) {
  __shared__ int wsum[MASK_T / 64];
  __shared__ uint32_t wbyte[MASK_T / 64];
  const int fw = blockIdx.x * MASK_T + (int)threadIdx.x;
  const int i0 = fw << 5;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t m = 0;
  if (i0 + 32 <= d.N) {
    const uint4* c4 = reinterpret_cast<const uint4*>(d.code + i0);
    const uint4 a = c4[0], b = c4[1];
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((v[q] >> (8 * k)) & 0xFFu) m |= 1u << (4 * q + k);
  } else {
    for (int k = 0; i0 + k < d.N && k < 32; ++k)
      if (d.code[i0 + k]) m |= 1u << k;
  }
  if (i0 < d.N) {
    d.imask[fw] = m;
    d.rmask[fw] = 0u;
  }
  // coarse word fw >> 3: four bits (one per 8 agents) from each of its 8 fine words
  uint32_t cb = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if ((m >> (8 * g)) & 0xFFu) cb |= 1u << g;
  uint32_t coarse = cb << (4 * (fw & 7));
  coarse |= __shfl_xor(coarse, 1);
  coarse |= __shfl_xor(coarse, 2);
  coarse |= __shfl_xor(coarse, 4);
  const int w = fw >> 3;
  if ((fw & 7) == 0 && w < ((d.N + 255) >> 8)) d.cmask[w] = coarse;
  // super-coarse: bit (w & 63) of word w >> 6 = some agent of coarse word w infectious;
  // a wave holds 8 coarse words, a workgroup one super-coarse word
  const unsigned long long bl = __ballot((fw & 7) == 0 && coarse != 0u);
  uint32_t byte = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) byte |= (uint32_t)((bl >> (8 * k)) & 1ull) << k;
  // one atomic per workgroup (a single counter: the fewer the better)
  int ninf = __builtin_popcount(m);
  for (int o = 32; o > 0; o >>= 1) ninf += __shfl_xor(ninf, o);
  if (lane == 0) {
    wsum[wv] = ninf;
    wbyte[wv] = byte;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    unsigned long long sc = 0ull;
    for (int q = 0; q < MASK_T / 64; ++q) {
      t += wsum[q];
      sc |= (unsigned long long)wbyte[q] << (8 * q);
    }
    if (t) atomicAdd(d.ninf, t);
    if ((int)blockIdx.x < d.nsc) d.scmask[blockIdx.x] = sc;
  }
}

// A frontier day: few enough agents infectious (k_mask's count) that the force of
// infection sums only the rows that hold an infectious source.
__device__ __forceinline__ bool sparse_day(const Dev& d) {
  return d.sparse_div > 0 && (int64_t)*d.ninf * d.sparse_div <= (int64_t)d.N;
}

// ---- vaccination plan ----------------------------------------------------------------
// The day's plan of replicate r: from the day the prevalence latch fires, the capacity
// goes to the priority classes in order; bstar is the first class that does not fit
// entirely and quota the doses left for it, filled by ascending agent id: each tile's
// first rank inside bstar is the number of bstar agents in the replicate's earlier
// tiles.  Replicates of at most 2048 tiles take one workgroup (k_vplan); larger ones
// are summed per segment of 256 tiles (k_vsum), planned (k_vplan_seg) and ranked per
// segment (k_vtile), so that no workgroup walks a replicate's tiles one round after
// another.

// Latched today: the latch fired before, or yesterday's prevalence reaches the trigger.
__device__ __forceinline__ bool latched_today(const Dev& d, int r) {
  if (d.latch[r]) return true;
  const long long* pc = d.prev_counts + (size_t)r * ABM_NC;
  const long long ei = pc[ABM_C_E] + pc[ABM_C_I] + pc[ABM_C_HOSP] + pc[ABM_C_ICU];
  return (double)ei >= d.vacc_trigger * (double)d.rep[r].n;
}

// bstar and quota from the class totals (thread 0); writes the plan and the latch.
__device__ __forceinline__ void make_plan(const Dev& d, int r, const long long* tot, int* plan) {
  const RepInfo& ri = d.rep[r];
  long long rem = ri.cap;
  int bstar = NBUCKET, quota = 0;
  for (int b = 0; b < NBUCKET; ++b) {
    if (tot[b] > rem) {
      bstar = b;
      quota = (int)rem;
      break;
    }
    rem -= tot[b];
  }
  plan[0] = bstar;
  plan[1] = quota;
  d.vplan[2 * r] = bstar;
  d.vplan[2 * r + 1] = quota;
  d.latch[r] = 1;
}

__global__ __launch_bounds__(TILE) void k_vplan(Dev d) {
  __shared__ int tot[TILE / 64][NBUCKET];
  __shared__ int plan[2];
  __shared__ int wsum[TILE / 64];
  __shared__ int carry;
  const int r = blockIdx.x;
  const RepInfo& ri = d.rep[r];
  if (!latched_today(d, r)) {
    if (threadIdx.x == 0) {
      d.vplan[2 * r] = -1;
      d.vplan[2 * r + 1] = 0;
    }
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int b = 0; b < NBUCKET; ++b) {
    int s = 0;
    for (int k = threadIdx.x; k < ri.ntiles; k += TILE) s += d.vhist[(size_t)(ri.tile0 + k) * NBUCKET + b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) tot[wv][b] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t[NBUCKET];
    for (int b = 0; b < NBUCKET; ++b) {
      t[b] = 0;
      for (int q = 0; q < TILE / 64; ++q) t[b] += tot[q][b];
    }
    make_plan(d, r, t, plan);
    carry = 0;
  }
  __syncthreads();
  const int bstar = plan[0];
  if (bstar >= NBUCKET) return;
  for (int k0 = 0; k0 < ri.ntiles; k0 += TILE) {
    const int k = k0 + threadIdx.x;
    const int v = k < ri.ntiles ? d.vhist[(size_t)(ri.tile0 + k) * NBUCKET + bstar] : 0;
    int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int wb = 0;
    for (int q = 0; q < wv; ++q) wb += wsum[q];
    if (k < ri.ntiles) d.vtile_base[ri.tile0 + k] = carry + wb + inc - v;
    __syncthreads();
    if (threadIdx.x == TILE - 1) carry += wb + inc;
    __syncthreads();
  }
}

// Segment s (tiles 256 s ..) of replicate r: its class totals, one lane per tile.
__global__ __launch_bounds__(TILE) void k_vsum(Dev d) {
  __shared__ int tot[TILE / 64][NBUCKET];
  const int s = blockIdx.x, r = blockIdx.y;
  const RepInfo& ri = d.rep[r];
  if (256 * s >= ri.ntiles || !latched_today(d, r)) return;
  const int k = 256 * s + (int)threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int* h = d.vhist + (size_t)(ri.tile0 + k) * NBUCKET;
#pragma unroll
  for (int b = 0; b < NBUCKET; ++b) {
    int v = k < ri.ntiles ? h[b] : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) tot[wv][b] = v;
  }
  __syncthreads();
  if (threadIdx.x < NBUCKET) {
    const int b = threadIdx.x;
    d.vpart[((size_t)r * d.vseg + s) * NBUCKET + b] = (tot[0][b] + tot[1][b]) + (tot[2][b] + tot[3][b]);
  }
}

// The plan of replicate r from its segments' totals, and each segment's first rank in
// bstar (a scan over the segments, 1024 at a time).
__global__ __launch_bounds__(1024) void k_vplan_seg(Dev d) {
  __shared__ long long tot[1024 / 64][NBUCKET];
  __shared__ int plan[2];
  __shared__ int wsum[1024 / 64];
  __shared__ int carry;
  const int r = blockIdx.x;
  const RepInfo& ri = d.rep[r];
  if (!latched_today(d, r)) {
    if (threadIdx.x == 0) {
      d.vplan[2 * r] = -1;
      d.vplan[2 * r + 1] = 0;
    }
    return;
  }
  const int nseg = (ri.ntiles + 255) / 256;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int* vp = d.vpart + (size_t)r * d.vseg * NBUCKET;
  for (int b = 0; b < NBUCKET; ++b) {
    long long v = 0;
    for (int s = threadIdx.x; s < nseg; s += 1024) v += vp[(size_t)s * NBUCKET + b];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) tot[wv][b] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t[NBUCKET];
    for (int b = 0; b < NBUCKET; ++b) {
      t[b] = 0;
      for (int q = 0; q < 1024 / 64; ++q) t[b] += tot[q][b];
    }
    make_plan(d, r, t, plan);
    carry = 0;
  }
  __syncthreads();
  const int bstar = plan[0];
  if (bstar >= NBUCKET) return;
  for (int s0 = 0; s0 < nseg; s0 += 1024) {
    const int s = s0 + (int)threadIdx.x;
    const int v = s < nseg ? vp[(size_t)s * NBUCKET + bstar] : 0;
    int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int wb = 0;
    for (int q = 0; q < wv; ++q) wb += wsum[q];
    if (s < nseg) d.vsegbase[(size_t)r * d.vseg + s] = carry + wb + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += wb + inc;
    __syncthreads();
  }
}

// Each tile's first rank in bstar: its segment's base plus a scan inside the segment.
__global__ __launch_bounds__(TILE) void k_vtile(Dev d) {
  __shared__ int wsum[TILE / 64];
  const int s = blockIdx.x, r = blockIdx.y;
  const RepInfo& ri = d.rep[r];
  const int bstar = d.vplan[2 * r];
  if (256 * s >= ri.ntiles || bstar < 0 || bstar >= NBUCKET) return;
  const int k = 256 * s + (int)threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = k < ri.ntiles ? d.vhist[(size_t)(ri.tile0 + k) * NBUCKET + bstar] : 0;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0;
  for (int q = 0; q < wv; ++q) wb += wsum[q];
  if (k < ri.ntiles) d.vtile_base[ri.tile0 + k] = d.vsegbase[(size_t)r * d.vseg + s] + wb + inc - v;
}

// ---- force of infection: lambda_j = coef[a_j] * sum_{e in row j} w_e * Atab[code[src_e]]
// A tile of 256 rows streams its contiguous edge range through LDS in chunks of CHUNK
// edges: the column loads and the infectious-mask tests are spread over all lanes; the
// weight and the code byte are read only for infectious sources (the others add +0).
// Each lane then sums its own row left to right (FP32, canonical order) from LDS, so
// the result does not depend on CHUNK or on how tiles map to workgroups (the grid may
// be one workgroup per tile or a persistent grid striding over the tiles).
template <int CHUNK, bool LDSMASK, int G>
__global__ __launch_bounds__(TILE * G) void k_message(Dev d) {
  // G tiles per workgroup (one per 256-lane group) share one LDS copy of the mask.
  // Sources are read four at a time (16-byte loads from a 4-aligned start) and each
  // lane issues U of those loads, then the mask lookups of all 4U sources, before it
  // uses any of them, so that many independent loads are in flight.
  typedef int v4i __attribute__((ext_vector_type(4)));
  constexpr int U = CHUNK / (TILE * 4) < 4 ? CHUNK / (TILE * 4) : 4;
  constexpr int NE = 4 * U;
  static_assert(CHUNK == TILE * NE, "a chunk is one round of loads");
  constexpr int NW = CHUNK / 32;
  extern __shared__ unsigned long long scm[];        // super-coarse mask (LDSMASK)
  __shared__ float atab[ATAB];
  __shared__ float term_[G][CHUNK];                  // written only where the source is infectious
  __shared__ uint32_t nzb_[G][2][NW];                // which terms of the chunk are written
  __shared__ uint32_t ninf_[G][TILE / 64];
  __shared__ int nch_max;
  const int grp = threadIdx.x / TILE, tid = threadIdx.x % TILE;
  float* term = term_[grp];
  if (threadIdx.x < ATAB) atab[threadIdx.x] = d.atab[threadIdx.x];
  if (*d.flags || sparse_day(d)) return;
  const float wh = d.w_h, wo = d.w_o, wr = d.w_r;   // network factors, in registers
  if (LDSMASK)
    for (int q = threadIdx.x; q < d.nsc; q += TILE * G) scm[q] = d.scmask[q];
  for (int q = threadIdx.x; q < G * 2 * NW; q += TILE * G) (&nzb_[0][0][0])[q] = 0u;
  int par = 0;
  for (int tb = blockIdx.x * G; tb < d.ntiles; tb += gridDim.x * G) {
    const int tix = tb + grp;
    const bool tv = tix < d.ntiles;
    const int4 tl = tv ? d.tiles[tix] : make_int4(0, 0, 0, 0);
    const int i = tl.y + tid;
    const bool live = tv && i < tl.z;
    const int e0 = tv ? d.row_ptr[tl.y] : 0, e1 = tv ? d.row_ptr[tl.z] : 0;
    const int rs = live ? d.row_ptr[i] : 0, re = live ? d.row_ptr[i + 1] : 0;
    const int a0 = e0 & ~3;
    const int nch = e1 > a0 ? (e1 - a0 + CHUNK - 1) / CHUNK : 0;
    float sum = 0.f;
    uint32_t infected_edges = 0;
    __syncthreads();
    if (threadIdx.x == 0) nch_max = 0;
    __syncthreads();
    if (tid == 0) atomicMax(&nch_max, nch);
    __syncthreads();
    const int nc = nch_max;
    // a chunk is one round of loads (CHUNK = TILE * NE); the next chunk's sources are
    // loaded before the current chunk's mask lookups
    v4i vn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = (u * TILE + tid) * 4;
      vn[u] = 0 < nch && k < min(CHUNK, e1 - a0) ? __builtin_nontemporal_load((const v4i*)(d.col + a0 + k))
                                               : v4i{0, 0, 0, 0};
    }
    for (int ci = 0; ci < nc; ++ci, par ^= 1) {
      const int c0 = a0 + ci * CHUNK;
      const int cn = ci < nch ? min(CHUNK, e1 - c0) : 0;
      uint32_t* nz = nzb_[grp][par];
      v4i v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = vn[u];
      if (ci + 1 < nch) {
        const int c1 = c0 + CHUNK, cn1 = min(CHUNK, e1 - c1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = (u * TILE + tid) * 4;
          vn[u] = k < cn1 ? __builtin_nontemporal_load((const v4i*)(d.col + c1 + k)) : v4i{0, 0, 0, 0};
        }
      }
      for (int kb = 0; kb < cn; kb += TILE * NE) {
        uint32_t src[NE];
        bool hit[NE];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const int k = kb + (u * TILE + tid) * 4 + l;
            const uint32_t x = (uint32_t)v[u][l] & COL_AGENT;
            src[4 * u + l] = x < (uint32_t)d.N ? x : 0u;
            hit[4 * u + l] = k < cn && c0 + k >= e0;
          }
        if (LDSMASK) {
#pragma unroll
          for (int q = 0; q < NE; ++q)
            hit[q] = hit[q] && ((scm[src[q] >> 14] >> ((src[q] >> 8) & 63u)) & 1ull);
        }
        uint32_t cw[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) cw[q] = hit[q] ? d.cmask[src[q] >> 8] : 0u;
#pragma unroll
        for (int q = 0; q < NE; ++q) hit[q] = (cw[q] >> ((src[q] >> 3) & 31u)) & 1u;
#pragma unroll
        for (int q = 0; q < NE; ++q) cw[q] = hit[q] ? d.imask[src[q] >> 5] : 0u;
        float wv[NE];
        uint32_t cd[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          hit[q] = (cw[q] >> (src[q] & 31u)) & 1u;
          wv[q] = col_weight((uint32_t)v[q >> 2][q & 3], wh, wo, wr);
          cd[q] = hit[q] ? (uint32_t)d.code[src[q]] : 0u;
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
          if (hit[q]) {
            const int k = kb + ((q >> 2) * TILE + tid) * 4 + (q & 3);
            term[k] = wv[q] * atab[cd[q]];
            atomicOr(&nz[k >> 5], 1u << (k & 31));
            ++infected_edges;
          }
        }
      }
      __syncthreads();
      const int lo = max(rs, c0) - c0, hi = min(re, c0 + cn) - c0;
      for (int wd = lo >> 5; lo < hi && wd <= (hi - 1) >> 5; ++wd) {
        uint32_t bits = nz[wd];
        const int b0 = wd << 5;
        if (lo > b0) bits &= ~0u << (lo - b0);
        if (hi < b0 + 32) bits &= (1u << (hi - b0)) - 1u;
        while (bits) {
          sum += term[b0 + __builtin_ctz(bits)];
          bits &= bits - 1u;
        }
      }
      for (int q = tid; q < NW; q += TILE) nzb_[grp][par ^ 1][q] = 0u;
      __syncthreads();
    }
    if (live) d.lambda[i] = d.rep[tl.x].coef[d.age[i]] * sum;
    for (int o = 32; o > 0; o >>= 1) infected_edges += __shfl_xor(infected_edges, o);
    if ((tid & 63) == 0) ninf_[grp][tid >> 6] = infected_edges;
    __syncthreads();
    if (tid == 0 && tv)
      d.tile_counts[(size_t)tix * TILE_NC + ABM_C_INF_EDGES] =
          ninf_[grp][0] + ninf_[grp][1] + ninf_[grp][2] + ninf_[grp][3];
  }
}

// Wave-private variant: a workgroup of 16 waves takes 4 tiles, each wave the 64 rows
// of a quarter tile, whose edges are one contiguous range.  A wave streams its range
// in WCH-edge chunks through its own LDS terms and bitmap, so only the wave itself
// touches them and no workgroup barrier is needed until the tiles' counts.
template <int WCH>
__global__ __launch_bounds__(1024) void k_message_w(Dev d) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  constexpr int U = WCH / 256;                      // 16-byte loads a lane per chunk
  constexpr int NE = 4 * U;
  constexpr int NW = WCH / 32;
  extern __shared__ unsigned long long scm[];       // super-coarse mask
  __shared__ float atab[ATAB];
  __shared__ float term_[16][WCH];
  __shared__ uint32_t nzb_[16][NW];
  __shared__ uint32_t ninf_[4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* term = term_[wv];
  uint32_t* nz = nzb_[wv];
  if (threadIdx.x < ATAB) atab[threadIdx.x] = d.atab[threadIdx.x];
  if (*d.flags || sparse_day(d)) return;
  const float wh = d.w_h, wo = d.w_o, wr = d.w_r;   // network factors, in registers
  // A wave's row bounds, row pointers and coefficient for the next workgroup iteration
  // (and the tile bounds for the one after) are loaded while the current one runs, and
  // are taken into registers before its stores: a load used only after a store waits
  // for that store as well.
  struct Rows {
    int r0, r1, e0, e1, rs, re, rep, age;
  };
  const int stride = gridDim.x * 4;
  auto tile_of = [&](int tb) {
    const int tix = tb + (wv >> 2);
    return tix < d.ntiles ? d.tiles[tix] : make_int4(0, 0, 0, 0);
  };
  auto rows_of = [&](const int4& tl) {          // every index clamped into its array
    Rows r;
    r.r0 = tl.y + 64 * (wv & 3);
    r.r1 = min(tl.z, r.r0 + 64);
    const int i = min(r.r0 + lane, d.N - 1);
    r.e0 = d.row_ptr[min(r.r0, d.N)];
    r.e1 = d.row_ptr[min(max(r.r1, 0), d.N)];
    r.rs = d.row_ptr[i];
    r.re = d.row_ptr[i + 1];
    r.rep = tl.x;
    // the aligned word holding the age byte (the age array is padded to 256 bytes);
    // the byte is extracted only where it is used
    r.age = (int)*reinterpret_cast<const uint32_t*>(d.age + (i & ~3));
    return r;
  };
  auto hold = [&](const Rows& r, const int4& t) {
    asm volatile("" ::"v"(r.r0), "v"(r.r1), "v"(r.e0), "v"(r.e1), "v"(r.rs), "v"(r.re), "v"(r.age));
    asm volatile("" ::"v"(t.x), "v"(t.y), "v"(t.z));
  };
  for (int q = threadIdx.x; q < d.nsc; q += 1024) scm[q] = d.scmask[q];
  Rows nxt = rows_of(tile_of(blockIdx.x * 4));
  int4 tln = tile_of(blockIdx.x * 4 + stride);
  hold(nxt, tln);
  __syncthreads();
  for (int tb = blockIdx.x * 4; tb < d.ntiles; tb += stride) {
    const int tix = tb + (wv >> 2);
    const Rows R = nxt;
    nxt = rows_of(tln);
    tln = tile_of(tb + 2 * stride);
    if (threadIdx.x < 4) ninf_[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t infected_edges = 0;
    if (tix < d.ntiles) {
      const int r0 = R.r0, r1 = R.r1;
      if (r0 < r1) {
        const int i = r0 + lane;
        const bool live = i < r1;
        const int e0 = R.e0, e1 = R.e1;
        const int rs = live ? R.rs : 0, re = live ? R.re : 0;
        float sum = 0.f;
        for (int c0 = e0 & ~3; c0 < e1; c0 += WCH) {
          const int cn = min(WCH, e1 - c0);
          for (int q = lane; q < NW; q += 64) nz[q] = 0u;
          v4i v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = (u * 64 + lane) * 4;
            v[u] = k < cn ? __builtin_nontemporal_load((const v4i*)(d.col + c0 + k)) : v4i{0, 0, 0, 0};
          }
          uint32_t src[NE];
          bool hit[NE];
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              const int k = (u * 64 + lane) * 4 + l;
              const uint32_t x = (uint32_t)v[u][l] & COL_AGENT;
              src[4 * u + l] = x < (uint32_t)d.N ? x : 0u;
              hit[4 * u + l] = k < cn && c0 + k >= e0 &&
                               ((scm[src[4 * u + l] >> 14] >> ((src[4 * u + l] >> 8) & 63u)) & 1ull);
            }
          uint32_t cw[NE];
#pragma unroll
          for (int q = 0; q < NE; ++q) cw[q] = hit[q] ? d.cmask[src[q] >> 8] : 0u;
#pragma unroll
          for (int q = 0; q < NE; ++q) hit[q] = (cw[q] >> ((src[q] >> 3) & 31u)) & 1u;
#pragma unroll
          for (int q = 0; q < NE; ++q) cw[q] = hit[q] ? d.imask[src[q] >> 5] : 0u;
          float wvv[NE];
          uint32_t cd[NE];
#pragma unroll
          for (int q = 0; q < NE; ++q) {
            hit[q] = (cw[q] >> (src[q] & 31u)) & 1u;
            wvv[q] = col_weight((uint32_t)v[q >> 2][q & 3], wh, wo, wr);
            cd[q] = hit[q] ? (uint32_t)d.code[src[q]] : 0u;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int q = 0; q < NE; ++q) {
            if (hit[q]) {
              const int k = ((q >> 2) * 64 + lane) * 4 + (q & 3);
              term[k] = wvv[q] * atab[cd[q]];
              atomicOr(&nz[k >> 5], 1u << (k & 31));
              ++infected_edges;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const int lo = max(rs, c0) - c0, hi = min(re, c0 + cn) - c0;
          for (int wd = lo >> 5; lo < hi && wd <= (hi - 1) >> 5; ++wd) {
            uint32_t bits = nz[wd];
            const int b0 = wd << 5;
            if (lo > b0) bits &= ~0u << (lo - b0);
            if (hi < b0 + 32) bits &= (1u << (hi - b0)) - 1u;
            while (bits) {
              sum += term[b0 + __builtin_ctz(bits)];
              bits &= bits - 1u;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
        hold(nxt, tln);
        if (live) d.lambda[i] = d.rep[R.rep].coef[((uint32_t)R.age >> (8 * (min(i, d.N - 1) & 3))) & 0xFFu] * sum;
      }
      for (int o = 32; o > 0; o >>= 1) infected_edges += __shfl_xor(infected_edges, o);
      if (lane == 0) atomicAdd(&ninf_[wv >> 2], infected_edges);
    }
    hold(nxt, tln);
    __syncthreads();
    if (threadIdx.x < 4 && tb + (int)threadIdx.x < d.ntiles)
      d.tile_counts[(size_t)(tb + threadIdx.x) * TILE_NC + ABM_C_INF_EDGES] = ninf_[threadIdx.x];
  }
}

// ---- frontier force of infection ------------------------------------------------------
// With few infectious agents, most rows hold no infectious source and sum to +0.  The
// graph is symmetric (a household pair or a drawn contact gives an edge in each
// direction), so the rows that hold infectious agent j are exactly the agents listed in
// row j: k_mark flags them from the infectious agents' own rows, k_front_list lists the
// flagged rows, and k_message_front sums each, term by term in edge order as the
// streaming kernels do, so lambda and the infectious-edge counts are bitwise the same.
__global__ __launch_bounds__(TILE) void k_mark(Dev d) {
  if (*d.flags || !sparse_day(d)) return;
  const int w = blockIdx.x * TILE + threadIdx.x;
  if (w >= (d.N + 31) >> 5) return;
  uint32_t m = d.imask[w];
  while (m) {
    const int j = (w << 5) + __builtin_ctz(m);
    m &= m - 1u;
    const int e1 = d.row_ptr[j + 1];
    for (int e = d.row_ptr[j]; e < e1; ++e) {
      const uint32_t i = (uint32_t)d.col[e] & COL_AGENT;
      if (i < (uint32_t)d.N) atomicOr(&d.rmask[i >> 5], 1u << (i & 31u));
    }
  }
}

// Every lambda is set to +0 (as the streaming sum of no terms gives; the flagged rows
// are overwritten next), every tile's infectious-edge count starts at 0, and the flagged
// rows are listed.  A wave takes 256 agents, four a lane; its flagged rows join list
// (group of 256 mod FRONT_NB) with one atomic for the wave's slots: a single list would
// put every wave's atomic on one address.
__global__ __launch_bounds__(TILE) void k_front_list(Dev d) {
  if (*d.flags || !sparse_day(d)) return;
  const int gid = blockIdx.x * TILE + threadIdx.x, nthr = gridDim.x * TILE;
  for (int q = gid; q < d.ntiles; q += nthr) d.tile_counts[(size_t)q * TILE_NC + ABM_C_INF_EDGES] = 0u;
  const int lane = threadIdx.x & 63;
  const int ngrp = (d.N + 255) >> 8;
  for (int g = gid >> 6; g < ngrp; g += nthr >> 6) {         // uniform per wave
    const int i0 = (g << 8) + 4 * lane;
    if (i0 + 3 < d.N) {
      *reinterpret_cast<float4*>(d.lambda + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      for (int k = i0; k < d.N; ++k) d.lambda[k] = 0.f;
    }
    const uint32_t f = i0 < d.N ? (d.rmask[i0 >> 5] >> (i0 & 31)) & 0xFu : 0u;
    const int c = __builtin_popcount(f);
    int inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    const int total = __shfl(inc, 63);
    if (total == 0) continue;
    const int list = g & (FRONT_NB - 1);
    int base = 0;
    if (lane == 0) base = atomicAdd(&d.nwork[list], total);
    base = __shfl(base, 0);
    int32_t* out = d.work + (size_t)list * d.work_cap + base + inc - c;
    for (int k = 0, m = 0; k < 4; ++k)
      if ((f >> k) & 1u) out[m++] = i0 + k;
  }
}

// A workgroup per list, one lane per flagged row: its edges four at a time (sources, then their mask words,
// then the codes of the infectious ones), the terms added in edge order.
__global__ __launch_bounds__(TILE) void k_message_front(Dev d) {
  __shared__ float atab[ATAB];
  if (threadIdx.x < ATAB) atab[threadIdx.x] = d.atab[threadIdx.x];
  if (*d.flags || !sparse_day(d)) return;
  __syncthreads();
  const float wh = d.w_h, wo = d.w_o, wr = d.w_r;
  const int n = d.nwork[blockIdx.x];               // workgroup b takes list b
  const int32_t* list = d.work + (size_t)blockIdx.x * d.work_cap;
  for (int q = threadIdx.x; q < n; q += TILE) {
    const int i = list[q];
    const int rs = d.row_ptr[i], re = d.row_ptr[i + 1];
    float sum = 0.f;
    uint32_t hits = 0;
    for (int e = rs; e < re; e += 4) {
      uint32_t x[4], s[4], m[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = e + u < re ? (uint32_t)d.col[e + u] : 0u;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s[u] = (x[u] & COL_AGENT) < (uint32_t)d.N ? (x[u] & COL_AGENT) : 0u;
        m[u] = e + u < re ? d.imask[s[u] >> 5] : 0u;
      }
      uint32_t cd[4];
      bool hit[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        hit[u] = (m[u] >> (s[u] & 31u)) & 1u;
        cd[u] = hit[u] ? (uint32_t)d.code[s[u]] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (hit[u]) {
          // the streaming kernels round each term to FP32 before adding it: no fused
          // multiply-add here either
#pragma clang fp contract(off)
          const float term = col_weight(x[u], wh, wo, wr) * atab[cd[u]];
          sum += term;
          ++hits;
        }
    }
    // the row's replicate: the last one starting at or before i
    int lo = 0, hi = d.R - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.rep[mid].start <= i) lo = mid;
      else hi = mid - 1;
    }
    const RepInfo& ri = d.rep[lo];
    d.lambda[i] = ri.coef[d.age[i]] * sum;
    if (hits) atomicAdd(&d.tile_counts[(size_t)(ri.tile0 + (i - ri.start) / TILE) * TILE_NC + ABM_C_INF_EDGES], hits);
  }
}

// ---- fused day step ---------------------------------------------------------------
__global__ __launch_bounds__(TILE) void k_fused(Dev d) {
  __shared__ int wpre[TILE / 64];
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const bool live = i < tl.z;
  const RepInfo& ri = d.rep[tl.x];
  const int t = *d.day;
  AgentState a;
  int age = 0;
  if (live) {
    a = d.state[i];
    age = d.age[i];
  }
  bool dose1 = false, dose2 = false;
  if (d.vacc_on) {
    const int bstar = d.vplan[2 * tl.x];
    const int quota = d.vplan[2 * tl.x + 1];
    if (bstar >= 0) {
      const int b = live ? vacc_bucket(d, a, t, age, ri.delay) : NBUCKET;
      bool dose = b < bstar;
      const bool inb = (b == bstar);
      // rank among this tile's members of the partial class, in agent order
      const unsigned long long m = __ballot(inb);
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
      if (lane == 0) wpre[wv] = __popcll(m);
      __syncthreads();
      int before = 0;
      for (int q = 0; q < wv; ++q) before += wpre[q];
      if (inb && bstar < NBUCKET) {
        const int rank = d.vtile_base[blockIdx.x] + before + __popcll(m & lt);
        dose = rank < quota;
      }
      if (dose) {
        if (a.vacc == 0) {
          a.vacc = 1;
          a.d1 = (int16_t)t;
          dose1 = true;
        } else {
          a.vacc = 2;
          a.d2 = (int16_t)t;
          dose2 = true;
        }
      }
    }
  }
  bool is_new = false, near = false, tested = false, notified = false;
  if (live) {
    const uint32_t loc = (uint32_t)(i - ri.start);
    bool immune = false;
    if (a.d1 != ABM_NEVER) {
      const uint4 bv = philox(loc, (uint32_t)(int)a.d1, ri.stream, P_VACC << 24, d.key0, d.key1);
      const float uv = u01(bv.x);
      immune = (t >= (int)a.d1 + d.dose_lag && uv < d.eff1) ||
               (a.d2 != ABM_NEVER && t >= (int)a.d2 + d.dose_lag && uv < d.eff2);
    }
    const uint4 b = philox(loc, (uint32_t)t, ri.stream, P_AGENT << 24, d.key0, d.key1);
    const int st0 = a.stage;
    const int tau = t - (int)a.t_exp;
    if (st0 == ABM_STAGE_S) {
      if (!immune || d.immune_asym) {
        const double p = -expm1(-(double)d.lambda[i] * (double)d.dt);
        const double u = (double)u01(b.x);
        if (u < p) {
          a.t_exp = (int16_t)t;
          is_new = true;
          if (d.course_on)
            course_infect(d, a, loc, t, ri.stream, age, immune);
          else
            a.stage = ABM_STAGE_E;
        }
        near = fabs(u - p) <= 1e-6;
      }
    } else if (d.course_on) {
      if ((int)a.t_next == t) course_step(d, a, loc, t, ri.stream, age);
    } else if (st0 == ABM_STAGE_E) {
      if (tau == d.e_days) a.stage = ABM_STAGE_I;
    } else if (st0 == ABM_STAGE_I) {
      if (tau == d.e_days + d.i_days) a.stage = u01(b.y) < d.p_death[age] ? ABM_STAGE_M : ABM_STAGE_R;
    }
    // contacts of today's positive app users that use the app themselves and are not in
    // quarantine are told to test tomorrow
    if (d.den_on && ((d.den_mask[i >> 5] >> (i & 31)) & 1u) && t >= (int)a.q_until)
      notified = app_user(d, loc, ri.stream);
    if ((d.test_rate > 0.f || d.den_on) && st0 != ABM_STAGE_M && t >= (int)a.q_until && !(a.flags & 1)) {
      bool sel = u01(b.z) < d.test_rate;
      if (!sel && d.den_on && (a.flags & 4)) {    // notified yesterday: tests with the compliance
        const uint4 b2 = philox(loc, (uint32_t)t, ri.stream, P_AGENT2 << 24, d.key0, d.key1);
        sel = u01(b2.z) < d.den_compliance;
      }
      if (sel) {
        tested = true;
        const bool infected = st0 != ABM_STAGE_S && st0 != ABM_STAGE_R && st0 != ABM_STAGE_M;
        const bool pos = infected && u01(b.w) < d.sens;
        a.flags = (uint8_t)(1 | (pos ? 2 : 0));
        a.test_day = (int16_t)t;
      }
    }
    a.flags = (uint8_t)((a.flags & ~4) | (notified ? 4 : 0));
    d.state[i] = a;
  }
  const int st = live ? (int)a.stage : -1;
  const bool v[13] = {st == ABM_STAGE_S, stage_e(st), stage_i(st), st == ABM_STAGE_R, st == ABM_STAGE_M,
                      st == ABM_STAGE_HOSP, st == ABM_STAGE_ICU, is_new, tested, dose1, dose2, near,
                      notified};
  const int sl[13] = {ABM_C_S, ABM_C_E, ABM_C_I, ABM_C_R, ABM_C_M, ABM_C_HOSP, ABM_C_ICU, ABM_C_NEW,
                      ABM_C_TESTS, ABM_C_DOSE1, ABM_C_DOSE2, ABM_C_NEAR, ABM_C_NOTIFIED};
  block_count_store<13>(v, sl, d.tile_counts + (size_t)blockIdx.x * TILE_NC);
}

// ---- end of day: tile counts -> per-replicate counts -> trajectory ----------------
// Integer sums, so the grouping does not change them.  Part (s, r) sums every fseg-th
// block of 256 tile rows of replicate r; one lane per count then adds the parts.
__global__ __launch_bounds__(TILE) void k_fin_part(Dev d) {
  __shared__ unsigned long long part[TILE / 64][ABM_NC];
  const int s = blockIdx.x, r = blockIdx.y;
  const RepInfo& ri = d.rep[r];
  unsigned long long acc[ABM_NC];
#pragma unroll
  for (int c = 0; c < ABM_NC; ++c) acc[c] = 0ull;
  for (int k = s * TILE + threadIdx.x; k < ri.ntiles; k += d.fseg * TILE) {
    const uint4* row = (const uint4*)(d.tile_counts + (size_t)(ri.tile0 + k) * TILE_NC);
    const uint4 a = row[0], b = row[1], c = row[2], e = row[3];
    const uint32_t v[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, e.x, e.y, e.z, e.w};
#pragma unroll
    for (int q = 0; q < ABM_NC; ++q) acc[q] += v[q];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < ABM_NC; ++c) {
    unsigned long long v = acc[c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) part[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < ABM_NC) {
    const int c = threadIdx.x;
    d.fin_part[((size_t)r * d.fseg + s) * TILE_NC + c] = part[0][c] + part[1][c] + part[2][c] + part[3][c];
  }
}

__global__ __launch_bounds__(64) void k_finalize(Dev d) {
  const int r = blockIdx.x;
  const RepInfo& ri = d.rep[r];
  const int t = *d.day;
  const bool ok = *d.flags == 0;
  if (threadIdx.x < ABM_NC) {
    const int c = threadIdx.x;
    long long v = 0;
    for (int q = 0; q < d.fseg; ++q) v += (long long)d.fin_part[((size_t)r * d.fseg + q) * TILE_NC + c];
    if (c == ABM_C_EDGES) v = ok ? (long long)d.row_ptr[ri.start + ri.n] - d.row_ptr[ri.start] : 0;
    if (c == ABM_C_INF_EDGES && !ok) v = 0;
    if (t < d.T) d.traj[((size_t)t * d.R + r) * ABM_NC + c] = v;
    d.prev_counts[(size_t)r * ABM_NC + c] = v;
  }
}

__global__ void k_advance_day(Dev d) { *d.day = *d.day + 1; }

// Small replicates (at most 2048 tiles): one workgroup per replicate adds its tile rows
// in one part, writes the day's counts as k_finalize does, and the last workgroup to
// finish advances the day (every workgroup has read it by then).
__global__ __launch_bounds__(TILE) void k_fin_one(Dev d) {
  __shared__ unsigned long long part[TILE / 64][ABM_NC];
  const int r = blockIdx.x;
  const RepInfo& ri = d.rep[r];
  const int t = *d.day;
  const bool ok = *d.flags == 0;
  // the day's edge count, loaded before the tile rows so that its latency overlaps theirs
  long long edges = 0;
  if (threadIdx.x == ABM_C_EDGES) edges = (long long)d.row_ptr[ri.start + ri.n] - d.row_ptr[ri.start];
  unsigned long long acc[ABM_NC];
#pragma unroll
  for (int c = 0; c < ABM_NC; ++c) acc[c] = 0ull;
  for (int k = threadIdx.x; k < ri.ntiles; k += TILE) {
    const uint4* row = (const uint4*)(d.tile_counts + (size_t)(ri.tile0 + k) * TILE_NC);
    const uint4 a = row[0], b = row[1], c = row[2], e = row[3];
    const uint32_t v[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, e.x, e.y, e.z, e.w};
#pragma unroll
    for (int q = 0; q < ABM_NC; ++q) acc[q] += v[q];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < ABM_NC; ++c) {
    unsigned long long v = acc[c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) part[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < ABM_NC) {
    const int c = threadIdx.x;
    long long v = (long long)(part[0][c] + part[1][c] + part[2][c] + part[3][c]);
    if (c == ABM_C_EDGES) v = ok ? edges : 0;
    if (c == ABM_C_INF_EDGES && !ok) v = 0;
    if (t < d.T) d.traj[((size_t)t * d.R + r) * ABM_NC + c] = v;
    d.prev_counts[(size_t)r * ABM_NC + c] = v;
  }
  if (threadIdx.x == 0 && atomicAdd(d.fin_done, 1) == (int)gridDim.x - 1) {
    *d.fin_done = 0;
    *d.day = t + 1;
  }
}

// ---- initial state: everyone susceptible, seeds exposed on day -1 --------------------
__global__ __launch_bounds__(TILE) void k_init_state(Dev d) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= d.N) return;
  AgentState a;
  a.stage = ABM_STAGE_S;
  a.flags = 0;
  a.vacc = 0;
  a.course = 0;
  a.t_exp = ABM_NEVER;
  a.q_until = ABM_NEVER;
  a.test_day = ABM_NEVER;
  a.d1 = ABM_NEVER;
  a.d2 = ABM_NEVER;
  a.t_next = (int16_t)ABM_NEVER;
  d.state[i] = a;
  d.code[i] = 0;
  d.lambda[i] = 0.f;
}

__global__ void k_seed(Dev d, const int32_t* seeds, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = seeds[k];
  AgentState a = d.state[i];
  a.t_exp = -1;                          // exposed the day before day 0
  if (d.course_on) {
    int lo = 0, hi = d.R - 1;            // the seed's replicate
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.rep[mid].start <= i) lo = mid; else hi = mid - 1;
    }
    const RepInfo& ri = d.rep[lo];
    course_infect(d, a, (uint32_t)(i - ri.start), -1, ri.stream, d.age[i]);
  } else {
    a.stage = ABM_STAGE_E;
  }
  d.state[i] = a;
}

__global__ void k_zero_counts(Dev d) {
  for (int k = threadIdx.x; k < d.R * ABM_NC; k += blockDim.x) d.prev_counts[k] = 0;
}

// Stage counts of the current state into prev_counts (for the prevalence latch).
__global__ __launch_bounds__(TILE) void k_recount(Dev d) {
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const int st = i < tl.z ? (int)d.state[i].stage : -1;
  const bool v[7] = {st == ABM_STAGE_S, stage_e(st), stage_i(st), st == ABM_STAGE_R, st == ABM_STAGE_M,
                     st == ABM_STAGE_HOSP, st == ABM_STAGE_ICU};
  const int sl[7] = {ABM_C_S, ABM_C_E, ABM_C_I, ABM_C_R, ABM_C_M, ABM_C_HOSP, ABM_C_ICU};
  block_count_add<7>(v, sl, reinterpret_cast<unsigned long long*>(d.prev_counts) + (size_t)tl.x * ABM_NC);
}

__global__ void k_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint4 r = philox(ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3],
                         (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  out[4 * k] = r.x;
  out[4 * k + 1] = r.y;
  out[4 * k + 2] = r.z;
  out[4 * k + 3] = r.w;
}

__global__ void k_set_day(Dev d, int32_t day) { *d.day = day; }

// The day's graph (row pointers and columns) into its slot of the notification ring.
__global__ __launch_bounds__(TILE) void k_den_clear(Dev d) {
  const int nw = (d.N + 31) / 32;
  for (int k = blockIdx.x * TILE + threadIdx.x; k < nw; k += gridDim.x * TILE) d.den_mask[k] = 0u;
}

void launch_pre(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_pre, dim3(d.ntiles), dim3(TILE), 0, s, d);
}
void launch_mask(const Dev& d, hipStream_t s) {
  const int nfw = (d.N + 31) >> 5;
  hipLaunchKernelGGL(k_mask, dim3((nfw + MASK_T - 1) / MASK_T), dim3(MASK_T), 0, s, d);
}
void launch_vplan(const Dev& d, hipStream_t s) {
  if (d.vseg == 0) {
    hipLaunchKernelGGL(k_vplan, dim3(d.R), dim3(TILE), 0, s, d);
    return;
  }
  hipLaunchKernelGGL(k_vsum, dim3(d.vseg, d.R), dim3(TILE), 0, s, d);
  hipLaunchKernelGGL(k_vplan_seg, dim3(d.R), dim3(1024), 0, s, d);
  hipLaunchKernelGGL(k_vtile, dim3(d.vseg, d.R), dim3(TILE), 0, s, d);
}
// Message-kernel variants the autotuner chooses from: LDS chunk x grid shape x where
// the first mask level lives (L2, or LDS for persistent grids when it fits) x tiles per
// workgroup (four 256-lane groups share one LDS copy of the mask).
int message_variants() { return 33; }

void message_variant(const Dev& d, int v, int32_t* chunk, int32_t* grid, int32_t* shape) {
  static const int chunks[3] = {1024, 2048, 4096};
  const bool fits = (size_t)d.nsc * 8 <= SCMASK_LDS_MAX;
  if (v >= 27) {                                 // wave-private chunks, four tiles a workgroup
    const int w = v - 27;
    *chunk = w % 2 ? 512 : 256;
    *grid = std::min((d.ntiles + 3) / 4, 256 << (w / 2));
    *shape = fits ? 3 : 0;
    if (!fits) *grid = d.ntiles;
    return;
  }
  if (v >= 21) {                                 // four tiles per workgroup, mask in LDS
    const int w = v - 21;
    *chunk = chunks[w % 2];
    *grid = std::min((d.ntiles + 3) / 4, 256 << (w / 2));
    *shape = fits ? 2 : 0;
    if (!fits) *grid = d.ntiles;
    return;
  }
  const int sh = v / 3;                          // 0: a workgroup per tile; 1..6 persistent
  const int grids[4] = {d.ntiles, 256 * 4, 256 * 8, 256 * 16};
  *chunk = chunks[v % 3];
  *grid = std::min(d.ntiles, grids[sh == 0 ? 0 : 1 + (sh - 1) % 3]);
  *shape = (sh >= 4 && fits) ? 1 : 0;
}

template <int C>
static void launch_msg(const Dev& d, const dim3& g, hipStream_t s) {
  if constexpr (C <= 2048) {
    if (d.msg_shape == 2) {
      hipLaunchKernelGGL((k_message<C, true, 4>), g, dim3(TILE * 4), (size_t)d.nsc * 8, s, d);
      return;
    }
  }
  if (d.msg_shape >= 1)
    hipLaunchKernelGGL((k_message<C, true, 1>), g, dim3(TILE), (size_t)d.nsc * 8, s, d);
  else
    hipLaunchKernelGGL((k_message<C, false, 1>), g, dim3(TILE), 0, s, d);
}

void launch_message(const Dev& d, hipStream_t s) {
  if (d.sparse_div > 0) {            // both paths are launched; each runs only on its days
    hipLaunchKernelGGL(k_mark, dim3(((d.N + 31) / 32 + TILE - 1) / TILE), dim3(TILE), 0, s, d);
    hipLaunchKernelGGL(k_front_list, dim3(2048), dim3(TILE), 0, s, d);
    hipLaunchKernelGGL(k_message_front, dim3(FRONT_NB), dim3(TILE), 0, s, d);
  }
  const dim3 g(d.msg_grid > 0 ? d.msg_grid : d.ntiles);
  if (d.msg_shape == 3) {
    if (d.msg_chunk == 256)
      hipLaunchKernelGGL(k_message_w<256>, g, dim3(1024), (size_t)d.nsc * 8, s, d);
    else
      hipLaunchKernelGGL(k_message_w<512>, g, dim3(1024), (size_t)d.nsc * 8, s, d);
    return;
  }
  switch (d.msg_chunk) {
    case 1024: launch_msg<1024>(d, g, s); break;
    case 2048: launch_msg<2048>(d, g, s); break;
    default: launch_msg<4096>(d, g, s); break;
  }
}

void launch_fused(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_fused, dim3(d.ntiles), dim3(TILE), 0, s, d);
}
void launch_finalize(const Dev& d, hipStream_t s) {
  if (d.fin_one) {
    hipLaunchKernelGGL(k_fin_one, dim3(d.R), dim3(TILE), 0, s, d);
    return;
  }
  hipLaunchKernelGGL(k_fin_part, dim3(d.fseg, d.R), dim3(TILE), 0, s, d);
  hipLaunchKernelGGL(k_finalize, dim3(d.R), dim3(64), 0, s, d);
  hipLaunchKernelGGL(k_advance_day, dim3(1), dim3(1), 0, s, d);
}
void launch_init_state(const Dev& d, const int32_t* seeds, int64_t nseeds, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3((d.N + TILE - 1) / TILE), dim3(TILE), 0, s, d);
  if (nseeds > 0)
    hipLaunchKernelGGL(k_seed, dim3((unsigned)((nseeds + 255) / 256)), dim3(256), 0, s, d, seeds, nseeds);
}
void launch_recount(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_recount, dim3(d.ntiles), dim3(TILE), 0, s, d);
}
void launch_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, ctr, n, out);
}
void launch_den_clear(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_den_clear, dim3(256), dim3(TILE), 0, s, d);
}
void launch_set_day(const Dev& d, int32_t day, hipStream_t s) {
  hipLaunchKernelGGL(k_set_day, dim3(1), dim3(1), 0, s, d, day);
}

}  // namespace abm
