// Daily contact-graph builder (section 3, "Interaction Networks"): fixed households,
// workplace contacts and random contacts redrawn every day, laid out as a
// destination-sorted CSR with a canonical order inside each row:
//   [household members ascending]
//   [workplace contacts the agent drew, draw order][workplace contacts others drew, by initiator]
//   [random contacts the agent drew, draw order][random contacts others drew, by initiator]
// Each drawn contact is seen from both ends (symmetric graph).
//
// Kernels: count (Poisson draws + atomic in-degree) -> scan (row pointers and claim
// cursors) -> fill (own rows + claimed slots in partners' rows) -> canon (sort each
// received block by initiator, write its weights).  The Philox draws are recomputed in fill rather than
// stored: ALU is cheaper than a round trip of the partner list through HBM.
#include "abm_internal.h"

namespace abm {

// Contacts drawn by one agent in one network: draw q (1..k) uses flat lane q of the
// network's Philox stream, lane 0 giving the Poisson count k.  Partners are uniform
// over the other m - 1 members of the agent's workplace (or replicate):
//   partner = member[(pos + 1 + floor(x (m - 1) / 2^32)) mod m].
struct ContactGen {
  uint32_t loc, t, stream, purpose, k0, k1, m, pos;
  int base;              // first agent of the replicate (random network)
  int wp_lo;             // offset of the workplace in the member list
  bool rnd;
  uint4 blk;
  uint32_t blk_id;

  __device__ __forceinline__ int count(const uint32_t* T) {
    if (m < 2) return 0;
    blk = philox(loc, t, stream, purpose << 24, k0, k1);
    blk_id = 0;
    return poisson_k(T, blk.x);
  }
  __device__ __forceinline__ int partner(const Dev& d, int q) {
    const uint32_t b = (uint32_t)q >> 2;
    if (b != blk_id) {
      blk = philox(loc, t, stream, (purpose << 24) | b, k0, k1);
      blk_id = b;
    }
    const uint32_t x = lane4(blk, q & 3);
    const uint32_t off = (uint32_t)(((uint64_t)x * (uint64_t)(m - 1)) >> 32);
    uint32_t slot = pos + 1 + off;
    if (slot >= m) slot -= m;
    return rnd ? base + (int)slot : d.wp_members[wp_lo + (int)slot];
  }
};

__device__ __forceinline__ ContactGen occ_gen(const Dev& d, const StaticRec& sr, uint32_t loc,
                                              uint32_t t, uint32_t stream) {
  ContactGen g;
  g.loc = loc; g.t = t; g.stream = stream; g.purpose = P_OCC; g.k0 = d.key0; g.k1 = d.key1;
  g.m = sr.wp_n; g.pos = sr.wp_pos; g.base = 0; g.wp_lo = sr.wp_lo; g.rnd = false;
  return g;
}

__device__ __forceinline__ ContactGen rand_gen(const Dev& d, const RepInfo& ri, uint32_t loc,
                                               uint32_t t) {
  ContactGen g;
  g.loc = loc; g.t = t; g.stream = ri.stream; g.purpose = P_RAND; g.k0 = d.key0; g.k1 = d.key1;
  g.m = (uint32_t)ri.n; g.pos = loc; g.base = ri.start; g.wp_lo = 0; g.rnd = true;
  return g;
}

constexpr int CLAIM_BATCH = 8;   // contacts whose memory operations are issued together

// In-degree from the other ends: one atomic increment per contact at its partner.
__device__ __forceinline__ int count_contacts(const Dev& d, ContactGen& g, const uint32_t* T,
                                              uint32_t inc) {
  const int k = g.count(T);
  for (int q0 = 1; q0 <= k; q0 += CLAIM_BATCH) {
    int p[CLAIM_BATCH];
#pragma unroll
    for (int b = 0; b < CLAIM_BATCH; ++b) p[b] = (q0 + b <= k) ? g.partner(d, q0 + b) : -1;
#pragma unroll
    for (int b = 0; b < CLAIM_BATCH; ++b)
      if (p[b] >= 0) atomicAdd(&d.recv[p[b]], inc);
  }
  return k;
}

// Own block (partners in draw order) and one claimed slot in each partner's received
// block.  The claims of a batch are independent, so they are all in flight at once.
__device__ __forceinline__ int fill_contacts(const Dev& d, ContactGen& g, const uint32_t* T,
                                             int32_t* cursor, int own, int self, uint32_t net) {
  const int k = g.count(T);
  for (int q0 = 1; q0 <= k; q0 += CLAIM_BATCH) {
    int p[CLAIM_BATCH], slot[CLAIM_BATCH];
#pragma unroll
    for (int b = 0; b < CLAIM_BATCH; ++b) p[b] = (q0 + b <= k) ? g.partner(d, q0 + b) : -1;
#pragma unroll
    for (int b = 0; b < CLAIM_BATCH; ++b)
      if (p[b] >= 0) slot[b] = atomicAdd(&cursor[p[b]], 1);
#pragma unroll
    for (int b = 0; b < CLAIM_BATCH; ++b)
      if (p[b] >= 0) {
        d.col[own + q0 + b - 1] = (int32_t)col_word((uint32_t)p[b], net);
        d.col[slot[b]] = (int32_t)col_word((uint32_t)self, net);
      }
  }
  return k;
}

__global__ __launch_bounds__(TILE) void k_count(Dev d) {
  __shared__ uint32_t T[NPT * 64];
  for (int i = threadIdx.x; i < NPT * 64; i += TILE) T[i] = d.ptab[i];
  __syncthreads();
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  if (i >= tl.z) return;
  const RepInfo& ri = d.rep[tl.x];
  const uint32_t t = (uint32_t)(*d.day);
  const StaticRec sr = d.srec[i];
  const uint32_t loc = (uint32_t)(i - ri.start);
  ContactGen go = occ_gen(d, sr, loc, t, ri.stream);
  const int ko = count_contacts(d, go, T + sr.occ * 64, 1u << 16);
  ContactGen gr = rand_gen(d, ri, loc, t);
  const int kr = count_contacts(d, gr, T + (PT_AGE0 + sr.age) * 64, 1u);
  d.own[i] = (uint16_t)(ko | (kr << 8));
}

__device__ __forceinline__ uint32_t degree_of(const Dev& d, int i) {
  const uint32_t o = d.own[i], r = d.recv[i];
  return (uint32_t)d.hhn[i] - 1u + (o & 0xFFu) + (o >> 8) + (r >> 16) + (r & 0xFFFFu);
}

// Phase 1: per-block sums of the degrees (a block is SCAN_BLOCK agents; the loads go
// with consecutive lanes on consecutive agents).
__global__ __launch_bounds__(TILE) void k_scan1(Dev d) {
  __shared__ uint32_t red[TILE / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * TILE;
    if (i < d.N) {
      const uint32_t r = d.recv[i];
      if ((r & 0xFFFFu) == 0xFFFFu || (r >> 16) == 0xFFFFu) atomicOr(d.flags, FLAG_RECV_OVERFLOW);
      s += degree_of(d, (int)i);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < TILE / 64; ++k) t += red[k];
    d.scan_part[blockIdx.x] = (int64_t)t;
  }
}

// Phase 2: one workgroup turns the block sums into exclusive offsets; checks capacity.
__global__ __launch_bounds__(1024) void k_scan2(Dev d) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < d.nscan; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    const int64_t v = b < d.nscan ? d.scan_part[b] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < d.nscan) d.scan_part[b] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    d.scan_part[d.nscan] = carry;
    if (carry > d.ecap) atomicOr(d.flags, FLAG_CAPACITY);
  }
}

// Phase 3: row pointers and the claim cursors of the two received blocks.  Wave w of a
// block takes SCAN_ITEMS rounds of 64 consecutive agents: a wave scan per round, the
// round's total carried to the next, so loads and stores stay coalesced.
__global__ __launch_bounds__(TILE) void k_scan3(Dev d) {
  __shared__ uint32_t wsum[TILE / 64];
  if (*d.flags) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)wv * 64 * SCAN_ITEMS;
  uint32_t deg[SCAN_ITEMS];
  uint32_t tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = wbase + k * 64 + lane;
    deg[k] = i < d.N ? degree_of(d, (int)i) : 0u;
    tot += deg[k];
  }
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
  if (lane == 0) wsum[wv] = tot;
  __syncthreads();
  int64_t run = d.scan_part[blockIdx.x];
  for (int q = 0; q < wv; ++q) run += wsum[q];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    uint32_t inc = deg[k];
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    const int64_t i = wbase + k * 64 + lane;
    if (i < d.N) {
      const int rp = (int)(run + inc - deg[k]);
      d.row_ptr[i] = rp;
      if (!d.pb_on) {            // claim cursors of the claim-based builder
        const uint32_t o = d.own[i], r = d.recv[i];
        const int co = rp + (int)d.hhn[i] - 1 + (int)(o & 0xFFu);
        d.cur_occ[i] = co;
        d.cur_rand[i] = co + (int)(r >> 16) + (int)(o >> 8);
      }
    }
    run += __shfl(inc, 63);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) d.row_ptr[d.N] = (int)d.scan_part[d.nscan];
}

__global__ __launch_bounds__(TILE) void k_fill(Dev d) {
  __shared__ uint32_t T[NPT * 64];
  for (int i = threadIdx.x; i < NPT * 64; i += TILE) T[i] = d.ptab[i];
  __syncthreads();
  if (*d.flags) return;
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  if (i >= tl.z) return;
  const RepInfo& ri = d.rep[tl.x];
  const uint32_t t = (uint32_t)(*d.day);
  const StaticRec sr = d.srec[i];
  const uint32_t loc = (uint32_t)(i - ri.start);
  int pos = d.row_ptr[i];
  for (int m = sr.hh_lo; m < sr.hh_lo + (int)sr.hh_n; ++m) {
    if (m == i) continue;
    d.col[pos] = m;                               // household: network 0
    ++pos;
  }
  const int own_occ = pos;
  ContactGen go = occ_gen(d, sr, loc, t, ri.stream);
  const int ko = fill_contacts(d, go, T + sr.occ * 64, d.cur_occ, own_occ, i, 1u);
  const int own_rand = own_occ + ko + (int)(d.recv[i] >> 16);
  ContactGen gr = rand_gen(d, ri, loc, t);
  fill_contacts(d, gr, T + (PT_AGE0 + sr.age) * 64, d.cur_rand, own_rand, i, 2u);
}

// Insertion sort of a short received block by initiator id.  Every word of a block
// carries the same network bits, so signed order is initiator order.
__device__ __forceinline__ void sort_block(int32_t* c, int n) {
  for (int a = 1; a < n; ++a) {
    const int32_t v = c[a];
    int b = a - 1;
    while (b >= 0 && c[b] > v) {
      c[b + 1] = c[b];
      --b;
    }
    c[b + 1] = v;
  }
}

// Blocks of up to 16 ids are sorted in registers by a bitonic network (all indices
// compile-time constants); longer ones (rare: Poisson tail) fall back to insertion.
__device__ __forceinline__ void sort_small(int32_t* c, int n) {
  if (n <= 1) return;
  if (n > 16) {
    sort_block(c, n);
    return;
  }
  int32_t v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = k < n ? c[k] : 0x7FFFFFFF;
#pragma unroll
  for (int size = 2; size <= 16; size <<= 1)
#pragma unroll
    for (int stride = size / 2; stride > 0; stride >>= 1)
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int l = k ^ stride;
        if (l > k) {
          const bool up = (k & size) == 0;
          const int32_t a = v[k], b = v[l];
          if ((a > b) == up) {
            v[k] = b;
            v[l] = a;
          }
        }
      }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < n) c[k] = v[k];
}

__global__ __launch_bounds__(TILE) void k_canon(Dev d) {
  if (*d.flags) return;
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= d.N) return;
  const uint32_t o = d.own[i], r = d.recv[i];
  const int ro = (int)(r >> 16), rr = (int)(r & 0xFFFFu);
  const int a = d.row_ptr[i] + (int)d.hhn[i] - 1 + (int)(o & 0xFFu);
  sort_small(d.col + a, ro);
  const int b = a + ro + (int)(o >> 8);
  sort_small(d.col + b, rr);
}

// In-degree counters start from zero each day (the hard step clears them in k_pre).
__global__ __launch_bounds__(TILE) void k_clear_recv(Dev d) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i < d.N) d.recv[i] = 0u;
}

void launch_clear_recv(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_recv, dim3((d.N + TILE - 1) / TILE), dim3(TILE), 0, s, d);
}
void launch_count(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(d.ntiles), dim3(TILE), 0, s, d);
}
void launch_scan(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_scan1, dim3(d.nscan), dim3(TILE), 0, s, d);
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(1024), 0, s, d);
  hipLaunchKernelGGL(k_scan3, dim3(d.nscan), dim3(TILE), 0, s, d);
}
void launch_fill(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(d.ntiles), dim3(TILE), 0, s, d);
}
void launch_canon(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_canon, dim3((d.N + TILE - 1) / TILE), dim3(TILE), 0, s, d);
}

}  // namespace abm
