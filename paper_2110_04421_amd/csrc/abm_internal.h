// Internal definitions shared by the HIP kernels and the host runtime of libabm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/abm.h"

namespace abm {

constexpr int TILE = 256;          // agents per tile (one workgroup of 4 waves)
constexpr int ATAB = 64;           // days-since-exposure table size
constexpr int NPT = 32;            // Poisson tables: 23 occupations + 9 age groups
constexpr int PT_AGE0 = ABM_N_OCC; // first age-group table
constexpr int NBUCKET = 18;        // vaccination priority classes (dose x age group)
constexpr int SCAN_ITEMS = 8;      // degrees per thread in the row-pointer scan
constexpr int SCAN_BLOCK = TILE * SCAN_ITEMS;
constexpr int MSG_CHUNK = 4096;    // edges staged in LDS per step of the message kernel
constexpr int TILE_NC = 16;       // per-tile count row (ABM_NC slots, padded)
static_assert(ABM_NC <= TILE_NC, "count slots fit a tile row");
constexpr size_t SCMASK_LDS_MAX = 48 * 1024;   // largest LDS copy of the super-coarse mask
constexpr int PB_S1_CAP = 12288;  // entries of a batch staged in LDS by the level-1 scatter
constexpr int PB_HS_MAX = 4608;   // bound on digits x (batches a workgroup + 1): sizes the P1 LDS histograms
constexpr int SPARSE_DIV = 256;
constexpr int64_t FRONT_MIN_N = 1 << 20;   // smallest population that takes the frontier path
constexpr int FRONT_NB = 1024;     // lists of flagged rows (256-agent group mod FRONT_NB): spread counters    // frontier force of infection with <= N/256 infectious agents
constexpr int WIN = 16;            // soft-mode exposure history ring (>= e_days + i_days + 1)

enum Purpose : uint32_t { P_AGENT = 0, P_AGENT2 = 1, P_VACC = 2, P_OCC = 3, P_RAND = 4, P_COURSE = 5, P_APP = 6 };

enum DevFlag : int32_t { FLAG_CAPACITY = 1, FLAG_RECV_OVERFLOW = 2 };

// Per-agent static data, 16 bytes.
struct StaticRec {
  int32_t hh_lo;      // first member of the household
  uint8_t hh_n;       // household size
  uint8_t age;
  uint8_t occ;
  uint8_t pad;
  int32_t wp_lo;      // offset of the workplace in wp_members (0 if none)
  uint16_t wp_pos;    // position in the workplace
  uint16_t wp_n;      // workplace size (0 if none)
};
static_assert(sizeof(StaticRec) == 16, "StaticRec is 16 bytes");

struct AgentState {
  uint8_t stage, flags, vacc, course;
  int16_t t_exp, q_until, test_day, d1, d2, t_next;
};
static_assert(sizeof(AgentState) == 16, "AgentState is 16 bytes");

// Per-replicate data (device copy).
struct RepInfo {
  int32_t start, n;         // agents [start, start + n)
  uint32_t stream;          // Philox stream word
  int32_t delay;            // dose-2 delay
  int64_t cap;              // daily doses
  int32_t tile0, ntiles;    // tiles of this replicate
  float coef[ABM_N_AGE];    // fl(fl(R * kappa) * S_a)
  float R;
  float S[ABM_N_AGE];
  float rk;                 // fl(R * kappa)
  int32_t pad[2];
};

// Everything a kernel needs, passed by value.
struct Dev {
  int32_t N, R, ntiles, T;
  int64_t ecap;
  uint32_t key0, key1;
  int32_t e_days, i_days, qdays, test_delay, dose_lag, vacc_on, strategy, mode;
  float w_h, w_o, w_r, dt, test_rate, sens, dropout, eff1, eff2, gtau, kappa;
  double vacc_trigger;
  float p_death[ABM_N_AGE];
  int8_t vrank[2][ABM_N_AGE];   // priority class of (dose 1|2, age group)
  int32_t course_on;            // eleven-stage course instead of SEIRM
  int32_t immune_asym;          // vaccine protection: asymptomatic infection, not none
  int32_t straight;             // relaxed mode: hard sample forward, relaxed derivative back
  float cprob[5][ABM_N_AGE];    // course: p_asym, p_severe, p_hosp, p_icu, p_die
  int32_t dur_shift[ABM_N_DUR];
  const uint32_t* dtab;         // [ABM_N_DUR][64] Poisson thresholds of the durations' extra days
  int32_t test_dmin, test_dmax; // result turnaround range (days)
  int32_t den_on, den_window;   // digital exposure notification
  float den_adoption, den_compliance;
  int32_t* ring_rp;             // [den_window][ring_rstride] row pointers of the last days' graphs
  int32_t* ring_col;            // [den_window][ring_cstride] their columns
  int64_t ring_rstride, ring_cstride;  // slot strides (elements); day t's graph is slot t % ring_n
  int32_t ring_n;               // graph slots: den_window (notification), the checkpoint
                                // interval (relaxed mode: the reverse sweep reuses the
                                // segment's graphs), else 1 (no ring)
  uint32_t* den_mask;           // [(N+31)/32] contacts of today's positive app users

  const RepInfo* rep;
  const int4* tiles;            // {rep, start, end, tile index}
  const StaticRec* srec;
  const uint8_t* age;
  const uint8_t* hhn;
  const int32_t* wp_members;
  const float* atab;            // [ATAB]
  const uint32_t* ptab;         // [NPT][64]

  AgentState* state;
  uint8_t* code;
  uint32_t* imask;              // bit i: agent i infectious today (code != 0)
  uint32_t* cmask;              // bit g: one of agents [8g, 8g + 8) infectious today
  unsigned long long* scmask;   // bit g: one of agents [256g, 256g + 256) infectious today
  int32_t nsc;                  // words of scmask
  float* lambda;

  uint16_t* own;                // k_occ | k_rand << 8 (drawn by the agent)
  uint32_t* recv;               // received occ << 16 | received rand
  int32_t* row_ptr;             // [N+1]
  int32_t* cur_occ;             // claim cursors into the received blocks
  int32_t* cur_rand;
  int32_t* col;                 // [E] source agent | network << 30 (col_agent, col_weight)
  int64_t* scan_part;           // [nscan + 1]
  int32_t nscan;

  int32_t* vhist;               // [ntiles][NBUCKET]
  int32_t* vplan;               // [R][2] partial class, quota in it
  int32_t* vtile_base;          // [ntiles]
  uint8_t* latch;               // [R]
  int32_t vseg;                 // segments of 256 tiles per replicate; 0: one workgroup plans a replicate
  int32_t* vpart;               // [R][vseg][NBUCKET] class totals per segment
  int32_t* vsegbase;            // [R][vseg] first rank of each segment in the partial class

  uint32_t* tile_counts;            // [ntiles][TILE_NC] each day's per-tile counts
  unsigned long long* fin_part;     // [R][fseg][TILE_NC] partial sums of the tile rows
  int32_t fseg, fin_one;     // fin_one: one launch per day reduces the counts (k_fin_one)
  long long* prev_counts;           // [R][ABM_NC]
  long long* traj;                  // [T][R][ABM_NC]
  int32_t* day;
  int32_t* fin_done;        // replicates whose day k_fin_one (k_soft_finalize) has closed
  int32_t* flags;

  // partitioned graph builder (k_build.hip)
  // frontier path of the force of infection: on a day with at most N / sparse_div
  // infectious agents, only rows with an infectious source are summed (0: never)
  uint32_t* rmask;              // bit i: row i holds an infectious source today
  int32_t* ninf;                // infectious agents today (counted by k_mask)
  int32_t* work;                // [FRONT_NB][work_cap] the flagged rows, by 256-agent group mod FRONT_NB
  int32_t* nwork;               // [FRONT_NB] their numbers
  int32_t work_cap;             // agents of a list's tiles at most
  int32_t sparse_div;
  int32_t msg_chunk, msg_grid, msg_shape;     // message-kernel tiling (autotuned or default);
                                              // shape 0: one tile a workgroup, masks in L2;
                                              // 1: one tile, mask in LDS; 2: four tiles, mask in LDS
  // The partitioned builder numbers destinations by tile slot, tile * 256 + row in the
  // tile, so that a leaf of 2^lb slots (lb = 8 or 9) is one or two whole tiles.  Level-1
  // buckets hold 2^(lb + 8) slots and split into 256 leaves; pb_nlv leaves hold tiles.
  int32_t pb_on, pb_lb, pb_nb1, pb_nbatch, pb_bpw, pb_ngrid, pb_bcap, pb_s1_nparts, pb_maxch, pb_nleaf,
      pb_nlv, pb_asm_cap, pb_s1_cap, pb_rper;
  int64_t pb_ccap;          // room for received entries (contacts) per day
  int32_t* pb_hist1;        // [nb1][nbatch] + 1: histograms, then run offsets
  uint32_t* pb_own;         // [nbatch][pb_bcap] each batch's own draws (slots), agent order
  int2* pb_tbase;           // [ntiles] a tile's first entry in its batch's own list, count
  int64_t* pb_part;         // [s1_nparts + 1]
  int32_t* pb_bstart;       // [nb1 + 1]
  int32_t* pb_bchunk;       // [nb1 + 1] first chunk of each bucket
  int32_t* pb_nchunks;      // [1]
  int4* pb_chunks;          // [maxch] {bucket, begin, end, 0}
  int32_t* pb_hist2;        // [maxch][256] histogram, then run offsets
  int32_t* pb_leaf;         // [nb1 * 256 + 1] leaf starts
  // level-1 partition, 6 bytes an entry: with dib = slot within its level-1 bucket
  // (lb + 8 bits) and sh = lb - 8: b1h = dib >> sh,
  // b1w = initiator | (dib & (2^sh - 1)) << 27 | network << 31
  uint16_t* pb_b1h;         // [ccap]
  uint32_t* pb_b1w;         // [ccap]
  // leaves: (row within the leaf (lb bits) | network << 15, initiator)
  uint2* pb_buf2;           // [ccap]
  int32_t pb_sh;
  int32_t* pb_tdeg;         // [ntiles] household and own edges of a tile's rows
  int32_t* pb_tstart;       // [nlv] a leaf's first edge within its group of 1024 leaves
  int64_t* pb_tpart;        // [nlv / 1024 + 1] first edge of each group; [last] = total
  int32_t pb_ntgrp;         // groups of 1024 leaves

  // soft mode
  float* s;            // susceptible mass [N]
  float* ehist;        // exposure mass ring [WIN][N], slot = day mod WIN
  float* inf;          // infectiousness [N]
  float* sigma;        // sum_e w * inf[src] of the day [N]
  float* soft_inc;     // [R][T] relaxed incidence
  float* seg_sigma;    // [seg][N] recompute buffers of a checkpoint segment
  float* seg_y;        // [seg][N]
  float* seg_s;        // [seg][N]
  float* ckpt;         // [nckpt][(WIN) + 1][N]
  float* s_bar;        // [N]
  float* ibar;         // [WIN][N] ring of adjoint of infectiousness, slot = day mod WIN
  float* vtmp;         // [N] coef * lambda_bar (message input of the transpose pass)
  float* lam_bar;      // [N]
  float* gtheta;       // [R][ABM_N_THETA] accumulated in float (per-tile partials reduced)
  float* gpart;        // [ntiles][ABM_N_THETA]
  const float* dL;     // [R][T] device copy of dL/d(incidence)
  int32_t seg;         // checkpoint interval
};

// ---- Philox4x32-10 (Salmon et al., SC'11) ------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32 -> 64-bit product per multiplier (a single v_mad_u64_u32 each)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t lane4(const uint4& b, int l) {
  return l == 0 ? b.x : (l == 1 ? b.y : (l == 2 ? b.z : b.w));
}

// A CSR column word: the source agent in the low 30 bits, its contact network in the
// top two (0 household, 1 occupation, 2 random).  The edge's weight is its network's
// factor, so no per-edge weight is stored.
constexpr uint32_t COL_AGENT = 0x3FFFFFFFu;
__device__ __forceinline__ uint32_t col_word(uint32_t agent, uint32_t net) { return agent | (net << 30); }
// (the three factors are passed as values: taken from the kernel arguments once, they
// stay in registers, and the choice is two selects, not a load)
__device__ __forceinline__ float col_weight(uint32_t c, float wh, float wo, float wr) {
  const uint32_t n = c >> 30;
  return n == 0u ? wh : (n == 1u ? wo : wr);
}

// (floor(x / 2^9) + 1/2) * 2^-23: odd multiples of 2^-24 in (0, 1), exact in FP32.
__device__ __forceinline__ float u01(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// Inverse-CDF Poisson count from a 32-bit word: #{k < 63 : T_k <= x}.
// #{k < 63 : T[k] <= x} for nondecreasing thresholds: the first k with T[k] > x, capped
// at 63, found in six uniform steps.
// Logical index of workgroup b in a grid of G workgroups, such that the workgroups the
// dispatcher places on one XCD (it deals them out b mod 8) take consecutive indices.
// Kernels whose neighbouring workgroups write into the same cache lines (the ends of
// short runs) use it, so that those lines are completed in one XCD's L2 instead of
// leaving two partial copies to be written back from two.
__host__ __device__ inline int xcd_block(int b, int G) {
  const int x = b & 7, q = b >> 3, base = G >> 3, rem = G & 7;
  return x * base + (x < rem ? x : rem) + q;
}

// The batches of workgroup b of a grid of G (groups of bpw batches, nbt batches in all)
// when one XCD's workgroups share its groups' batch range interleaved: the w-th of its
// c workgroups takes the range's batches w, w + c, w + 2c, ...  Returns the first
// batch, the stride and the count.
struct Interleave {
  int first, stride, count;
};
__host__ __device__ inline Interleave xcd_interleave(int b, int G, int bpw, int nbt) {
  const int x = b & 7, w = b >> 3, base = G >> 3, rem = G & 7;
  const int c = base + (x < rem ? 1 : 0), p = x * base + (x < rem ? x : rem);
  const int b0 = p * bpw, end = (p + c) * bpw < nbt ? (p + c) * bpw : nbt;
  const int n = end - b0 > w ? (end - b0 - w + c - 1) / c : 0;
  return Interleave{b0 + w, c, n};
}

__device__ __forceinline__ int poisson_k(const uint32_t* T, uint32_t x) {
  int lo = 0;
#pragma unroll
  for (int h = 32; h > 0; h >>= 1)
    if (lo + h <= 63 && T[lo + h - 1] <= x) lo += h;
  return lo;
}

// ---- kernel launchers (one per translation unit that owns the kernel) ---------------
void launch_pre(const Dev& d, hipStream_t s);
void launch_mask(const Dev& d, hipStream_t s);
void launch_vplan(const Dev& d, hipStream_t s);
void launch_count(const Dev& d, hipStream_t s);
void launch_clear_recv(const Dev& d, hipStream_t s);
void launch_scan(const Dev& d, hipStream_t s);
void launch_fill(const Dev& d, hipStream_t s);
void launch_canon(const Dev& d, hipStream_t s);
void launch_message(const Dev& d, hipStream_t s);
int message_variants();
void message_variant(const Dev& d, int v, int32_t* chunk, int32_t* grid, int32_t* shape);
void launch_fused(const Dev& d, hipStream_t s);
void launch_finalize(const Dev& d, hipStream_t s);
void launch_init_state(const Dev& d, const int32_t* seeds, int64_t nseeds, hipStream_t s);
void launch_recount(const Dev& d, hipStream_t s);
void launch_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t s);

// partitioned builder: named steps (for per-kernel timing) and one-time setup
int build_steps(const Dev& d);
const char* build_step_name(const Dev& d, int k);
void launch_build_step(const Dev& d, int k, hipStream_t s);
hipError_t prepare_build(const Dev& d);

// soft mode
void launch_soft_init(const Dev& d, const int32_t* seeds, int64_t nseeds, hipStream_t s);
void launch_soft_inf(const Dev& d, hipStream_t s);
void launch_soft_message(const Dev& d, const float* x, float* out, hipStream_t s);
void launch_soft_update(const Dev& d, int32_t seg_slot, hipStream_t s);
void launch_soft_finalize(const Dev& d, hipStream_t s);
void launch_soft_ckpt_save(const Dev& d, int32_t k, hipStream_t s);
void launch_soft_ckpt_load(const Dev& d, int32_t k, int32_t day, hipStream_t s);
void launch_adj_zero(const Dev& d, hipStream_t s);
void launch_adj_day(const Dev& d, int32_t t, int32_t seg_slot, hipStream_t s);
void launch_adj_ibar(const Dev& d, int32_t t, hipStream_t s);
void launch_adj_theta(const Dev& d, hipStream_t s);
void launch_den_clear(const Dev& d, hipStream_t s);   // end of day: notification marks consumed
void launch_set_day(const Dev& d, int32_t day, hipStream_t s);

}  // namespace abm
