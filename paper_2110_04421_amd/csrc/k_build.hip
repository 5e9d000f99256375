// Daily contact graph, partitioned builder.  Same CSR, same canonical order as the
// claim-based builder in k_graph.hip (section 3, "Interaction Networks"), built without
// global atomics and without random 4-byte scatters.  Destinations are numbered by tile
// slot (tile * 256 + row in the tile), so that the last level of the partition, a leaf
// of 2^LB slots (LB = 8 or 9), is one or two whole tiles of rows:
//
//   P1  gen         per batch of 4 tiles: draw every agent's contacts once (Philox, and
//                   the workplace-member loads), store the partners' slots in agent
//                   order in the batch's own list, keep the agent's counts and each
//                   tile's household + own edge count, histogram the partners by
//                   level-1 digit (slot >> (LB + 8)).
//   S1  scan        digit-major exclusive scan of the histograms -> each (digit, batch)
//                   run's offset; level-1 bucket bounds; chunk table.
//   P2  scatter-1   read the batch's own list, counting-sort its entries
//                   (slot, src | net) by digit in LDS, write each run contiguously
//                   as 6-byte entries (16-bit slot part, 32-bit source word).
//   P3  hist-2      per chunk of a level-1 bucket: histogram by leaf digit.
//   S2  scan-2      per bucket, digit-major scan -> run offsets; leaf bounds.
//   P4  scatter-2   entries into leaves.
//   S3  leaves      each leaf's first edge: a scan of the leaves' edge totals.
//   P5  rows        per leaf: count its entries per (row, network), row pointers, then
//                   each row: household, own occupation draws, received occupation,
//                   own random draws, received random, the received runs sorted by
//                   initiator in LDS.
// Every run written in P2/P4 leaves as consecutive lanes on consecutive addresses, and
// every random access of a per-edge scatter becomes an LDS access.
#include "abm_internal.h"

namespace abm {

constexpr int PB_THREADS = 1024;       // P1/P2 workgroup: one batch of 4 tiles at a time
constexpr int PB_UNROLL = 8;           // loads a lane issues before using them (P2, P3)
constexpr int PB_CHUNK = 8192;         // entries per level-2 chunk (sorted in LDS)
constexpr int PB_NB1_MAX = 1024;       // level-1 digits

// Contact generation: the same draws, in the same order, as k_graph.hip's.
struct Gen {
  uint32_t loc, t, stream, purpose, k0, k1, m, pos;
  int base, wp_lo;
  bool rnd;
  uint4 blk;
  __device__ __forceinline__ int count(const uint32_t* T) {
    if (m < 2) return 0;
    blk = philox(loc, t, stream, purpose << 24, k0, k1);
    return poisson_k(T, blk.x);
  }
  // f(q, partner) for q = 1..k in draw order (after count()).  The up-to-four partners
  // of one Philox block are computed, and their member-list loads issued, together.
  template <class F>
  __device__ __forceinline__ void each(const Dev& d, int k, F&& f) {
    for (int q0 = 0; q0 <= k; q0 += 4) {
      if (q0 > 0) blk = philox(loc, t, stream, (purpose << 24) | (uint32_t)(q0 >> 2), k0, k1);
      int p[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int q = q0 + l;
        p[l] = 0;
        if (q >= 1 && q <= k) {
          const uint32_t x = lane4(blk, l);
          const uint32_t off = (uint32_t)(((uint64_t)x * (uint64_t)(m - 1)) >> 32);
          uint32_t slot = pos + 1 + off;
          if (slot >= m) slot -= m;
          p[l] = rnd ? base + (int)slot : d.wp_members[wp_lo + (int)slot];
        }
      }
#pragma unroll
      for (int l = 0; l < 4; ++l)
        if (q0 + l >= 1 && q0 + l <= k) f(q0 + l, p[l]);
    }
  }
};

__device__ __forceinline__ Gen gen_occ(const Dev& d, const StaticRec& sr, uint32_t loc, uint32_t t,
                                       uint32_t stream) {
  Gen g;
  g.loc = loc; g.t = t; g.stream = stream; g.purpose = P_OCC; g.k0 = d.key0; g.k1 = d.key1;
  g.m = sr.wp_n; g.pos = sr.wp_pos; g.base = 0; g.wp_lo = sr.wp_lo; g.rnd = false;
  return g;
}
__device__ __forceinline__ Gen gen_rand(const Dev& d, const RepInfo& ri, uint32_t loc, uint32_t t) {
  Gen g;
  g.loc = loc; g.t = t; g.stream = ri.stream; g.purpose = P_RAND; g.k0 = d.key0; g.k1 = d.key1;
  g.m = (uint32_t)ri.n; g.pos = loc; g.base = ri.start; g.wp_lo = 0; g.rnd = true;
  return g;
}

// The generation pass streams the static records in and its own lists out with
// nontemporal accesses, so that they do not displace the workplace member lists that
// its partner draws read at random.
__device__ __forceinline__ StaticRec load_srec_nt(const StaticRec* p) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  const v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p));
  StaticRec r;
  __builtin_memcpy(&r, &v, sizeof(r));
  return r;
}

// Level-1 partition entry of (destination slot p, initiator | network << 31).
__device__ __forceinline__ void put_b1(const Dev& d, int pos, uint32_t p, uint32_t w) {
  const uint32_t dib = p & ((1u << (d.pb_lb + 8)) - 1u);
  d.pb_b1h[pos] = (uint16_t)(dib >> d.pb_sh);
  d.pb_b1w[pos] = w | ((dib & ((1u << d.pb_sh) - 1u)) << 27);
}

// ---- P1: draw each batch's contacts once --------------------------------------------
// 1024 lanes = one batch of 4 tiles of 256 agents; a workgroup takes pb_bpw batches.
// The batch's draws are staged in LDS in agent order (own workplace draws, then own
// random draws, each in draw order) and written contiguously to the batch's own list
// (pb_bcap entries a batch); pb_tbase[tile] is the tile's first entry in it and its
// number of entries.  The
// level-1 histograms (16-bit counters in LDS for all the workgroup's batches) are
// stored digit-major (digit * nbatch + batch) for the scan.
__global__ __launch_bounds__(PB_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void k_pb_gen(Dev d) {
  extern __shared__ __attribute__((aligned(16))) uint32_t stage[];   // [pb_bcap] draws, then [pb_bpw][nh2] histograms
  __shared__ uint32_t T[NPT * 64];
  __shared__ int wsum[PB_THREADS / 64], wdeg[PB_THREADS / 64];
  __shared__ int ntot;
  // two 16-bit counters a word (a batch has at most pb_bcap <= 24576 draws)
  const int nh2 = (d.pb_nb1 + 1) >> 1;
  uint32_t* hist = stage + d.pb_bcap;
  for (int k = threadIdx.x; k < NPT * 64; k += PB_THREADS) T[k] = d.ptab[k];
  for (int k = threadIdx.x; k < d.pb_bpw * nh2; k += PB_THREADS) hist[k] = 0u;
  __syncthreads();
  const uint32_t t = (uint32_t)(*d.day);
  const int s1 = d.pb_lb + 8;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = 0; j < d.pb_bpw; ++j) {
    const int bt = xcd_block(blockIdx.x, gridDim.x) * d.pb_bpw + j;
    if (bt >= d.pb_nbatch) break;
    uint32_t* h = hist + j * nh2;
    const int tix = bt * 4 + (tid >> 8);
    // across the barriers a lane keeps only its static record, replicate and the two
    // count blocks; the generators are rebuilt from them for the partner draws
    int i = 0, ko = 0, kr = 0, rep = 0;
    bool live = false;
    StaticRec sr{};
    uint4 bo = make_uint4(0u, 0u, 0u, 0u), br = bo;
    if (tix < d.ntiles) {
      const int4 tl = d.tiles[tix];
      i = tl.y + (tid & (TILE - 1));
      live = i < tl.z;
      rep = tl.x;
      if (live) {
        const RepInfo& ri = d.rep[rep];
        sr = load_srec_nt(d.srec + i);
        const uint32_t loc = (uint32_t)(i - ri.start);
        Gen go = gen_occ(d, sr, loc, t, ri.stream);
        ko = go.count(T + sr.occ * 64);
        bo = go.blk;
        Gen gr = gen_rand(d, ri, loc, t);
        kr = gr.count(T + (PT_AGE0 + sr.age) * 64);
        br = gr.blk;
        __builtin_nontemporal_store((uint16_t)(ko | (kr << 8)), d.own + i);
      }
    }
    const int c = ko + kr;
    int inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    // the row's household and own edges, summed over the tile for its first edge
    int hd = live ? (int)sr.hh_n - 1 + c : 0;
    for (int o = 32; o > 0; o >>= 1) hd += __shfl_xor(hd, o);
    if (lane == 63) wsum[wv] = inc;
    if (lane == 0) wdeg[wv] = hd;
    __syncthreads();
    int wb = 0;
    for (int q = 0; q < wv; ++q) wb += wsum[q];
    const int off = wb + inc - c;
    if (tid == PB_THREADS - 1) ntot = wb + inc;
    if ((tid & (TILE - 1)) == 0 && tix < d.ntiles) {    // the tile's own-list range
      int cnt = 0, dg = 0;
      for (int q = wv; q < wv + TILE / 64; ++q) {
        cnt += wsum[q];
        dg += wdeg[q];
      }
      d.pb_tbase[tix] = make_int2(off, cnt);
      d.pb_tdeg[tix] = dg;
    }
    __syncthreads();
    const int n = ntot;
    if (n > d.pb_bcap) {                     // more draws than the batch's room
      if (tid == 0) atomicOr(d.flags, FLAG_CAPACITY);
      return;
    }
    if (live) {
      const RepInfo& ri = d.rep[rep];
      const uint32_t loc = (uint32_t)(i - ri.start);
      Gen go = gen_occ(d, sr, loc, t, ri.stream);
      go.blk = bo;
      Gen gr = gen_rand(d, ri, loc, t);
      gr.blk = br;
      // partners are kept as tile slots (a partner is in its initiator's replicate)
      const int dl = (ri.tile0 << 8) - ri.start;
      go.each(d, ko, [&](int q, int p) {
        const int sl = p + dl;
        stage[off + q - 1] = (uint32_t)sl;
        const int dg = sl >> s1;
        atomicAdd(&h[dg >> 1], 1u << (16 * (dg & 1)));
      });
      gr.each(d, kr, [&](int q, int p) {
        const int sl = p + dl;
        stage[off + ko + q - 1] = (uint32_t)sl;
        const int dg = sl >> s1;
        atomicAdd(&h[dg >> 1], 1u << (16 * (dg & 1)));
      });
    }
    __syncthreads();
    // the batch's own list (it starts on a 16-byte boundary) in 16-byte stores
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    uint32_t* dst = d.pb_own + (size_t)bt * d.pb_bcap;
    const int nv = n >> 2;
    for (int v = tid; v < nv; v += PB_THREADS)
      __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(stage + 4 * v), reinterpret_cast<v4u*>(dst) + v);
    for (int k = 4 * nv + tid; k < n; k += PB_THREADS) __builtin_nontemporal_store(stage[k], dst + k);
    __syncthreads();
  }
  // the workgroup's histograms, digit-major: each digit's batches are consecutive
  const int bt0 = xcd_block(blockIdx.x, gridDim.x) * d.pb_bpw;
  const int nb = min(d.pb_bpw, d.pb_nbatch - bt0);
  for (int k = threadIdx.x; k < d.pb_nb1 * nb; k += PB_THREADS) {
    const int dg = k / nb, j = k - dg * nb;
    d.pb_hist1[(size_t)dg * d.pb_nbatch + bt0 + j] = (int)((hist[j * nh2 + (dg >> 1)] >> (16 * (dg & 1))) & 0xFFFFu);
  }
}

// ---- generic three-phase exclusive scan over a virtual index ----------------------------
// Level-1 order: q = digit * nbatch + batch, the storage order of hist1.
__device__ __forceinline__ int* h1_at(const Dev& d, int64_t q) { return d.pb_hist1 + q; }

static_assert(SCAN_ITEMS == 8, "the level-1 scan moves a lane's items as two 16-byte vectors");
__global__ __launch_bounds__(TILE) void k_pb_s1a(Dev d) {
  __shared__ int red[TILE / 64];
  const int64_t n = (int64_t)d.pb_nb1 * d.pb_nbatch;
  const int64_t q0 = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int s = 0;
  if (q0 + SCAN_ITEMS <= n) {                // whole: two 16-byte loads (q0 is a multiple of 8)
    const int4* p = reinterpret_cast<const int4*>(h1_at(d, q0));
    const int4 a = p[0], b = p[1];
    s = (a.x + a.y) + (a.z + a.w) + (b.x + b.y) + (b.z + b.w);
  } else {
    for (int k = 0; k < SCAN_ITEMS; ++k)
      if (q0 + k < n) s += *h1_at(d, q0 + k);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) d.pb_part[blockIdx.x] = (int64_t)(red[0] + red[1] + red[2] + red[3]);
}

// Exclusive scan of nparts block sums in place (one workgroup); total to parts[nparts].
// Each lane takes a contiguous run of ceil(nparts / 1024) sums; the run totals are
// scanned with wave shuffles and one barrier.
__global__ __launch_bounds__(1024) void k_pb_parts(int64_t* parts, int nparts) {
  __shared__ int64_t wsum[1024 / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = (nparts + 1023) / 1024, q0 = (int)threadIdx.x * per;
  int64_t s = 0;
  for (int k = 0; k < per; ++k)
    if (q0 + k < nparts) s += parts[q0 + k];
  int64_t inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int64_t run = 0, tot = 0;
  for (int q = 0; q < 1024 / 64; ++q) {
    if (q < wv) run += wsum[q];
    tot += wsum[q];
  }
  run += inc - s;
  for (int k = 0; k < per; ++k)
    if (q0 + k < nparts) {
      const int64_t v = parts[q0 + k];
      parts[q0 + k] = run;
      run += v;
    }
  if (threadIdx.x == 0) parts[nparts] = tot;
}

__global__ __launch_bounds__(TILE) void k_pb_s1c(Dev d) {
  __shared__ int wsum[TILE / 64];
  const int64_t n = (int64_t)d.pb_nb1 * d.pb_nbatch;
  const int64_t q0 = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int s = 0;
  const bool whole = q0 + SCAN_ITEMS <= n;   // two 16-byte loads and stores (q0 is a multiple of 8)
  if (whole) {
    const int4* p = reinterpret_cast<const int4*>(h1_at(d, q0));
    const int4 a = p[0], b = p[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = q0 + k < n ? *h1_at(d, q0 + k) : 0;
  }
  for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0;
  for (int k = 0; k < wv; ++k) wb += wsum[k];
  int64_t run = d.pb_part[blockIdx.x] + wb + inc - s;
  int ex[SCAN_ITEMS];
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    ex[k] = (int)run;
    run += v[k];
  }
  if (whole) {
    int4* p = reinterpret_cast<int4*>(h1_at(d, q0));
    p[0] = make_int4(ex[0], ex[1], ex[2], ex[3]);
    p[1] = make_int4(ex[4], ex[5], ex[6], ex[7]);
  } else {
    for (int k = 0; k < SCAN_ITEMS; ++k)
      if (q0 + k < n) *h1_at(d, q0 + k) = ex[k];
  }
}

// Bucket bounds and the level-2 chunk table (one workgroup; nb1 <= 1024).
__device__ void buckets_body(const Dev& d, int64_t total) {
  __shared__ int nch[PB_NB1_MAX + 1];
  __shared__ int wsum[1024 / 64];
  __shared__ int ok;
  const int b = threadIdx.x, lane = b & 63, wv = b >> 6;
  int start = 0, size = 0, n = 0;
  if (b < d.pb_nb1) {
    start = d.pb_hist1[(size_t)b * d.pb_nbatch];
    const int64_t end = b + 1 < d.pb_nb1 ? (int64_t)d.pb_hist1[(size_t)(b + 1) * d.pb_nbatch] : total;
    size = (int)(end - start);
    d.pb_bstart[b] = start;
    n = (size + PB_CHUNK - 1) / PB_CHUNK;
  }
  // each bucket's first chunk: a workgroup scan of the chunk counts
  int inc = n;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0, c = 0;
  for (int q = 0; q < 1024 / 64; ++q) {
    if (q < wv) wb += wsum[q];
    c += wsum[q];
  }
  if (b < d.pb_nb1) nch[b] = wb + inc - n;
  if (threadIdx.x == 0) {
    nch[d.pb_nb1] = c;
    *d.pb_nchunks = c;
    d.pb_hist1[(size_t)d.pb_nb1 * d.pb_nbatch] = (int)total;   // end of the last run
    d.pb_bstart[d.pb_nb1] = (int)total;
    ok = total <= d.pb_ccap && c <= d.pb_maxch;
    if (!ok) atomicOr(d.flags, FLAG_CAPACITY);
  }
  __syncthreads();
  if (b < d.pb_nb1 && ok) {
    for (int k = 0; k < nch[b + 1] - nch[b]; ++k) {
      const int c = nch[b] + k;
      const int lo = start + k * PB_CHUNK;
      d.pb_chunks[c] = make_int4(b, lo, min(lo + PB_CHUNK, start + size), 0);
    }
    d.pb_bchunk[b] = nch[b];
  }
  if (b == 0) d.pb_bchunk[d.pb_nb1] = nch[d.pb_nb1];
}

__global__ __launch_bounds__(1024) void k_pb_buckets(Dev d) { buckets_body(d, d.pb_part[d.pb_s1_nparts]); }

// The whole level-1 scan and the bucket table in one workgroup, where the histograms
// are few (small populations, whose day is bound by launches): each lane scans a
// contiguous run of at most PB_S1_ONE entries in place.
constexpr int PB_S1_ONE = 32;
__global__ __launch_bounds__(1024) void k_pb_s1_one(Dev d) {
  __shared__ int wsum[16];
  __shared__ int64_t tot;
  const int n = d.pb_nb1 * d.pb_nbatch;
  const int per = (n + 1023) / 1024;
  const int q0 = (int)threadIdx.x * per;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int s = 0;
  for (int k = 0; k < per; ++k)
    if (q0 + k < n) s += d.pb_hist1[q0 + k];
  int inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0;
  for (int q = 0; q < wv; ++q) wb += wsum[q];
  if (threadIdx.x == 1023) tot = (int64_t)(wb + inc);
  int run = wb + inc - s;
  for (int k = 0; k < per; ++k)
    if (q0 + k < n) {
      const int v = d.pb_hist1[q0 + k];
      d.pb_hist1[q0 + k] = run;
      run += v;
    }
  __syncthreads();                                   // the offsets are written
  buckets_body(d, tot);
}

// ---- P2: scatter into level-1 runs ---------------------------------------------------
// Per batch: its runs' offsets and sizes come from the scanned histograms.  The
// batch's own list is read with consecutive lanes on consecutive entries; an entry's
// initiator and network come from a 16-bit LDS tag that the initiator's lane wrote
// for each of its entries.  Entries are counting-sorted by digit into
// LDS and each run leaves as consecutive lanes on consecutive addresses; a batch with
// more than PB_S1_CAP entries writes each entry directly to its run.  The order inside
// a run is immaterial: the row pass orders fully.  The next batch's agent counts and
// the first rounds of its own list are loaded while the current batch is placed.
constexpr int PB_S1_PF = 10;           // own-list entries a lane loads for the next batch
__global__ __launch_bounds__(PB_THREADS) void k_pb_scatter1(Dev d) {
  __shared__ uint2 stage[PB_S1_CAP];
  __shared__ uint16_t tag[PB_S1_CAP];          // own-list entry -> initiator lane | network << 15
  __shared__ int gofs[PB_NB1_MAX], lst[PB_NB1_MAX], lcur[PB_NB1_MAX];
  __shared__ int aid[PB_THREADS];
  __shared__ int wsum[PB_THREADS / 64], wsum2[PB_THREADS / 64];
  __shared__ int nstage;
  if (*d.flags) return;
  const int s1 = d.pb_lb + 8;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nbt = d.pb_nbatch;
  // The batches of the workgroups that the dispatcher places on one XCD (it deals them
  // out blockIdx mod 8) form one range, and the w-th of its c workgroups takes batches
  // w, w + c, w + 2c, ... of it (xcd_interleave).  The workgroups running together on
  // an XCD then place neighbouring batches at the same time, so the line where one
  // batch's run for a digit ends and the next batch's begins is completed in that
  // XCD's L2 while both are written, instead of staying open there until the next
  // batch of the same workgroup.
  const Interleave il = xcd_interleave((int)blockIdx.x, (int)gridDim.x, d.pb_bpw, nbt);
  const int nb = il.count;
  // a batch's agent counts, its runs' offsets and the first PB_S1_PF rounds of its own
  // list are loaded one batch ahead, while the previous batch is sorted and written
  auto fetch = [&](int bt, int& i, uint32_t& o, uint32_t* pv, int& g, int& e) {
    const int tix = bt * 4 + (tid >> 8);
    i = -1;
    o = 0u;
    if (tix < d.ntiles) {
      const int4 tl = d.tiles[tix];
      const int a = tl.y + (tid & (TILE - 1));
      if (a < tl.z) {
        i = a;
        o = d.own[a];
      }
    }
    if (tid < d.pb_nb1) {              // run (digit, bt) ends where (digit, bt + 1) starts
      g = d.pb_hist1[(size_t)tid * nbt + bt];
      e = d.pb_hist1[(size_t)tid * nbt + bt + 1];
    }
    const uint32_t* src = d.pb_own + (size_t)bt * d.pb_bcap;
#pragma unroll
    for (int u = 0; u < PB_S1_PF; ++u) {
      const int k = u * PB_THREADS + tid;
      pv[u] = k < d.pb_bcap ? src[k] : 0u;
    }
  };
  int inx, gnx = 0, enx = 0;
  uint32_t onx, pvn[PB_S1_PF];
  if (nb > 0) fetch(il.first, inx, onx, pvn, gnx, enx);
  for (int j = 0; j < nb; ++j) {
    const int bt = il.first + j * il.stride;
    const int i = inx;
    const uint32_t o = onx;
    uint32_t pv[PB_S1_PF];
#pragma unroll
    for (int u = 0; u < PB_S1_PF; ++u) pv[u] = pvn[u];
    int cntv = 0;
    if (tid < d.pb_nb1) {
      gofs[tid] = gnx;
      cntv = enx - gnx;
    }
    const int ko = i >= 0 ? (int)(o & 0xFFu) : 0;
    const int c = i >= 0 ? ko + (int)(o >> 8) : 0;
    int inc = cntv, inc2 = c;
    for (int q = 1; q < 64; q <<= 1) {
      const int y = __shfl_up(inc, q), y2 = __shfl_up(inc2, q);
      if (lane >= q) {
        inc += y;
        inc2 += y2;
      }
    }
    if (lane == 63) {
      wsum[wv] = inc;
      wsum2[wv] = inc2;
    }
    __syncthreads();
    int wb = 0, wb2 = 0;
    for (int q = 0; q < wv; ++q) {
      wb += wsum[q];
      wb2 += wsum2[q];
    }
    if (tid < d.pb_nb1) {
      lst[tid] = wb + inc - cntv;
      lcur[tid] = wb + inc - cntv;
    }
    aid[tid] = i < 0 ? 0 : i;
    if (tid == PB_THREADS - 1) nstage = wb + inc;
    __syncthreads();
    const int nb_n = nstage;
    const bool staged = nb_n <= d.pb_s1_cap;
    // each agent's lane tags its own-list entries with its lane and their network
    if (staged) {
      const int ao = wb2 + inc2 - c;
      for (int q = 0; q < c; ++q) tag[ao + q] = (uint16_t)(tid | (q >= ko ? 0x8000 : 0));
    }
    __syncthreads();
    if (j + 1 < nb) fetch(bt + il.stride, inx, onx, pvn, gnx, enx);
    auto place = [&](int k, uint32_t p) {
      const uint32_t tg = tag[k];
      const uint32_t net = (tg & 0x8000u) << 16;
      const int dg = (int)(p >> s1);
      const int slot = atomicAdd(&lcur[dg], 1);
      stage[slot] = make_uint2(p, (uint32_t)aid[tg & 0x3FFu] | net);
    };
    if (staged) {
#pragma unroll
      for (int u = 0; u < PB_S1_PF; ++u) {
        const int k = u * PB_THREADS + tid;
        if (k >= nb_n) break;
        place(k, pv[u]);
      }
      const uint32_t* src = d.pb_own + (size_t)bt * d.pb_bcap;
      for (int kb = PB_S1_PF * PB_THREADS; kb < nb_n; kb += PB_THREADS * PB_UNROLL) {
        uint32_t qv[PB_UNROLL];
#pragma unroll
        for (int u = 0; u < PB_UNROLL; ++u) {
          const int k = kb + u * PB_THREADS + tid;
          qv[u] = k < nb_n ? src[k] : 0u;
        }
#pragma unroll
        for (int u = 0; u < PB_UNROLL; ++u) {
          const int k = kb + u * PB_THREADS + tid;
          if (k >= nb_n) break;
          place(k, qv[u]);
        }
      }
    } else if (i >= 0) {                           // a batch beyond the LDS room: direct
      const uint32_t* src = d.pb_own + (size_t)bt * d.pb_bcap + (wb2 + inc2 - c);
      for (int q = 0; q < c; ++q) {
        const uint32_t p = src[q];
        const int dg = (int)(p >> s1);
        const int slot = atomicAdd(&lcur[dg], 1);
        put_b1(d, gofs[dg] + slot - lst[dg], p, (uint32_t)i | (q >= ko ? 0x80000000u : 0u));
      }
    }
    __syncthreads();
    if (staged) {
      for (int k = tid; k < nb_n; k += PB_THREADS) {
        const uint2 x = stage[k];
        const int dg = (int)(x.x >> s1);
        put_b1(d, gofs[dg] + k - lst[dg], x.x, x.y);
      }
      __syncthreads();
    }
  }
}

// ---- P3: level-2 histograms per chunk -----------------------------------------------
__global__ __launch_bounds__(TILE) void k_pb_hist2(Dev d) {
  __shared__ int hist[256];
  if (*d.flags) return;
  const int c = blockIdx.x;
  if (c >= *d.pb_nchunks) return;
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int4 ch = d.pb_chunks[c];
  for (int eb = ch.y; eb < ch.z; eb += TILE * PB_UNROLL) {
    uint32_t x[PB_UNROLL];                       // all loads first, then their use
#pragma unroll
    for (int u = 0; u < PB_UNROLL; ++u) {
      const int e = eb + u * TILE + (int)threadIdx.x;
      x[u] = e < ch.z ? (uint32_t)d.pb_b1h[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < PB_UNROLL; ++u)
      if (eb + u * TILE + (int)threadIdx.x < ch.z) atomicAdd(&hist[(x[u] >> (d.pb_lb - d.pb_sh)) & 255u], 1);
  }
  __syncthreads();
  d.pb_hist2[(size_t)c * 256 + threadIdx.x] = hist[threadIdx.x];
}

// ---- S2: per bucket, digit-major exclusive scan of its chunks' histograms ------------
// Four lanes per digit, each taking a quarter of the digit's chunks: the lanes' runs
// follow the digit-major order, and at each step a wave reads 16 consecutive digits of
// 4 chunk rows.  Run sums, a workgroup scan of them, then the runs' offsets (two
// barriers; the histograms are read twice, the second time from cache).
constexpr int PB_S2_SCAN = 1024;
__global__ __launch_bounds__(PB_S2_SCAN) void k_pb_s2(Dev d) {
  __shared__ int wsum[PB_S2_SCAN / 64];
  if (*d.flags) return;
  const int b = blockIdx.x;
  const int c0 = d.pb_bchunk[b], nc = d.pb_bchunk[b + 1] - c0;
  const int base = d.pb_bstart[b];
  const int dg = threadIdx.x >> 2, part = threadIdx.x & 3;
  const int per = (nc + 3) >> 2;
  const int ca = min(nc, part * per), cb = min(nc, ca + per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int* h = d.pb_hist2 + ((size_t)c0 << 8) + dg;
  int s = 0;
  for (int cc = ca; cc < cb; ++cc) s += h[(size_t)cc << 8];
  int inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0;
  for (int k = 0; k < wv; ++k) wb += wsum[k];
  int run = base + wb + inc - s;
  if (part == 0) d.pb_leaf[((size_t)b << 8) + dg] = run;   // the digit's first chunk (or its empty run)
  for (int cc = ca; cc < cb; ++cc) {
    const int v = h[(size_t)cc << 8];
    h[(size_t)cc << 8] = run;
    run += v;
  }
  if (b == d.pb_nb1 - 1 && threadIdx.x == 0) d.pb_leaf[(size_t)d.pb_nb1 << 8] = d.pb_bstart[d.pb_nb1];
}

// ---- P4: scatter into leaves ---------------------------------------------------------
// The chunk is read once into registers (PB_S2_PER entries a lane), counting-sorted by
// leaf digit in LDS, and each leaf's part of the chunk leaves as one contiguous run of
// consecutive lanes.  The order inside a run is immaterial: the row pass orders fully.
constexpr int PB_S2_THREADS = 1024;
constexpr int PB_S2_PER = PB_CHUNK / PB_S2_THREADS;
__global__ __launch_bounds__(PB_S2_THREADS) void k_pb_scatter2(Dev d) {
  __shared__ uint2 sorted[PB_CHUNK];
  __shared__ int cnt[256], first[256];
  __shared__ int wsum[4];
  if (*d.flags) return;
  const int c = xcd_block(blockIdx.x, gridDim.x);
  if (c >= *d.pb_nchunks) return;
  const int4 ch = d.pb_chunks[c];
  const int n = ch.z - ch.y;
  const int tid = threadIdx.x;
  if (tid < 256) cnt[tid] = 0;
  __syncthreads();
  const int d2s = d.pb_lb - d.pb_sh;          // level-2 digit = (b1h >> d2s) & 255
  uint2 x[PB_S2_PER];                         // (b1h, b1w)
  int rank[PB_S2_PER];
#pragma unroll
  for (int j = 0; j < PB_S2_PER; ++j) {
    const int k = j * PB_S2_THREADS + tid;
    x[j] = k < n ? make_uint2((uint32_t)d.pb_b1h[ch.y + k], d.pb_b1w[ch.y + k]) : make_uint2(0u, 0u);
  }
#pragma unroll
  for (int j = 0; j < PB_S2_PER; ++j) {
    const int k = j * PB_S2_THREADS + tid;
    rank[j] = k < n ? atomicAdd(&cnt[(x[j].x >> d2s) & 255u], 1) : 0;
  }
  __syncthreads();
  const int v = tid < 256 ? cnt[tid] : 0;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if ((tid & 63) >= o) inc += y;
  }
  if (tid < 256 && (tid & 63) == 63) wsum[tid >> 6] = inc;
  __syncthreads();
  if (tid < 256) {
    int wb = 0;
    for (int q = 0; q < (tid >> 6); ++q) wb += wsum[q];
    first[tid] = wb + inc - v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PB_S2_PER; ++j) {
    const int k = j * PB_S2_THREADS + tid;
    if (k < n) sorted[first[(x[j].x >> d2s) & 255u] + rank[j]] = x[j];
  }
  __syncthreads();
  const int* off = d.pb_hist2 + (size_t)c * 256;
  const uint32_t lmask = (1u << d.pb_sh) - 1u, dmask = (1u << d.pb_lb) - 1u;
  for (int k = tid; k < n; k += PB_S2_THREADS) {
    const uint2 y = sorted[k];
    const int dg = (y.x >> d2s) & 255u;
    const int pos = off[dg] + (k - first[dg]);
    const uint32_t dib = (y.x << d.pb_sh) | ((y.y >> 27) & lmask);
    d.pb_buf2[pos] = make_uint2((dib & dmask) | ((y.y >> 31) << 15), y.y & 0x07FFFFFFu);
  }
}

// ---- S3: each leaf's first edge --------------------------------------------------
// A leaf's edges are its tiles' household and own edges (summed by P1) and its
// received entries; k_pb_tsum scans them within groups of PB_TGRP leaves and
// k_pb_parts scans the groups (not launched for a single group), so the row pointers
// come from about N/256 values, not N degrees.
constexpr int PB_TGRP = 1024;
__global__ __launch_bounds__(PB_TGRP) void k_pb_tsum(Dev d) {
  __shared__ int wsum[PB_TGRP / 64];
  if (*d.flags) return;
  const int L = blockIdx.x * PB_TGRP + (int)threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nt = 1 << (d.pb_lb - 8);
  int v = 0;
  if (L < d.pb_nlv) {
    v = d.pb_leaf[L + 1] - d.pb_leaf[L];
    for (int t = L * nt; t < min(L * nt + nt, d.ntiles); ++t) v += d.pb_tdeg[t];
  }
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wb = 0;
  for (int q = 0; q < wv; ++q) wb += wsum[q];
  if (L < d.pb_nlv) d.pb_tstart[L] = wb + inc - v;
  if (threadIdx.x == PB_TGRP - 1) {
    if (gridDim.x == 1) {                            // one group: its parts scanned here
      d.pb_tpart[0] = 0;
      d.pb_tpart[1] = (int64_t)(wb + inc);
    } else {
      d.pb_tpart[blockIdx.x] = (int64_t)(wb + inc);
    }
  }
}

// ---- P5: the rows of a leaf ------------------------------------------------------
// One workgroup per leaf of NT tiles (NT * 256 rows, one lane each; the tiles are
// consecutive rows of the CSR and consecutive ranges of one batch's own list).  The
// leaf's received entries (in no particular order) are read once into registers
// (pb_rper entries a lane, the rest read again from memory) and counted per (row,
// network) in LDS; with the household sizes and own counts these give the rows'
// degrees, whose scan after the leaf's first edge gives the row pointers.  Each lane
// lays out its row (household, own workplace draws, received workplace, own random
// draws, received random) in the LDS copy of the leaf's edge range: its household part
// and its own draws (read from the own list, where the rows' draws follow one another,
// so a wave reads one contiguous stretch), and the first position of each of its two
// received runs.  Each received entry takes the next position of its (row, network)
// run; each lane then sorts its two runs by initiator (they are short), and the edge
// range leaves with consecutive lanes on consecutive addresses.  A column word is the
// source id with the network in its top two bits.  A leaf with more edges than the LDS
// room is laid out in the column array itself.
constexpr int PB_ROWS_PER = 12;        // received entries a lane keeps in registers
__device__ __forceinline__ int slot_delta(const Dev& d, int tix) {   // slot - agent id
  const RepInfo& ri = d.rep[d.tiles[tix].x];
  return (ri.tile0 << 8) - ri.start;
}

template <int NT>
__global__ __launch_bounds__(NT * TILE) void k_pb_rows(Dev d) {
  constexpr int NR = NT * TILE;
  extern __shared__ int32_t scol[];                  // [cap] staged edges
  __shared__ int cur[2 * NR];                        // (row, network): received count, then next position
  __shared__ int wsum[NR / 64], wsum2[NR / 64], lsum[NR / 64];
  if (*d.flags) return;
  const int cap = d.pb_asm_cap;
  const int L = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  cur[tid] = 0;
  cur[tid + NR] = 0;
  const int t0 = L * NT, tix = t0 + tid / TILE;      // the leaf's first tile, this lane's tile
  const int2 tb0 = d.pb_tbase[t0];
  const uint32_t* ob = d.pb_own + (size_t)(t0 >> 2) * d.pb_bcap + tb0.x;   // the leaf's own range
  const int lo = d.pb_leaf[L], hi = d.pb_leaf[L + 1];
  const int nreg = min(hi - lo, d.pb_rper * NR);
  // the leaf's received entries, loaded with the rows' own data
  uint2 x[PB_ROWS_PER];
#pragma unroll
  for (int j = 0; j < PB_ROWS_PER; ++j) {
    const int k = j * NR + tid;
    x[j] = k < nreg ? d.pb_buf2[lo + k] : make_uint2(0u, 0u);
  }
  int i = 0, ko = 0, kr = 0;
  bool live = false;
  StaticRec sr{};
  if (tix < d.ntiles) {
    const int4 tl = d.tiles[tix];
    i = tl.y + (tid & (TILE - 1));
    live = i < tl.z;
    if (live) {
      const uint32_t o = d.own[i];
      ko = (int)(o & 0xFFu);
      kr = (int)(o >> 8);
      sr = d.srec[i];
    }
  }
  const int dl = tix < d.ntiles ? slot_delta(d, tix) : 0;   // this row's replicate
  auto rkey = [](uint32_t v) { return (int)(((v & (NR - 1)) << 1) | (v >> 15)); };
  // The leaf's first edge: from the leaf scan, or, with one group of leaves (where that
  // scan is not launched), the sum of the earlier leaves' edges, added up here.
  const bool own_sum = d.pb_ntgrp == 1;
  if (own_sum) {
    const int nt = 1 << (d.pb_lb - 8);
    int acc = 0;
    for (int l2 = tid; l2 < L; l2 += NR) {
      acc += d.pb_leaf[l2 + 1] - d.pb_leaf[l2];
      for (int t = l2 * nt; t < min(l2 * nt + nt, d.ntiles); ++t) acc += d.pb_tdeg[t];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) lsum[wv] = acc;
  }
  __syncthreads();                                   // counters cleared, leaf sums written
  int64_t b64 = 0;
  if (own_sum) {
    for (int q = 0; q < NR / 64; ++q) b64 += lsum[q];
  } else {
    b64 = d.pb_tpart[L / PB_TGRP] + d.pb_tstart[L];
  }
#pragma unroll
  for (int j = 0; j < PB_ROWS_PER; ++j)
    if (j * NR + tid < nreg) atomicAdd(&cur[rkey(x[j].x)], 1);
  for (int e = lo + nreg + tid; e < hi; e += NR) atomicAdd(&cur[rkey(d.pb_buf2[e].x)], 1);
  __syncthreads();
  // rows past a ragged tile's end have no slot a partner could draw: their counts are 0
  // the rows' degrees and own-draw counts, scanned together
  const int co = cur[2 * tid], cr = cur[2 * tid + 1];
  const int c = ko + kr;
  const int deg = live ? (int)sr.hh_n - 1 + c + co + cr : 0;
  int dinc = deg, inc = c;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(dinc, o), y2 = __shfl_up(inc, o);
    if (lane >= o) {
      dinc += y;
      inc += y2;
    }
  }
  if (lane == 63) {
    wsum[wv] = dinc;
    wsum2[wv] = inc;
  }
  __syncthreads();
  int dwb = 0, dtot = 0, wb = 0;
  for (int q = 0; q < NR / 64; ++q) {
    if (q < wv) {
      dwb += wsum[q];
      wb += wsum2[q];
    }
    dtot += wsum[q];
  }
  if (b64 + dtot > d.ecap) {                         // the same for every lane
    if (tid == 0) atomicOr(d.flags, FLAG_CAPACITY);
    return;
  }
  if (L == d.pb_nlv - 1 && tid == 0) d.row_ptr[d.N] = (int)(b64 + dtot);
  const int base = (int)b64, end = base + dtot;
  const int rp0 = base + dwb + dinc - deg;           // this row's first edge
  if (live) d.row_ptr[i] = rp0;
  const bool staged = end - base <= cap;
  // The layout, written once for each target so that the staged one addresses LDS
  // directly (a pointer that may be either would take the slower generic path).
  auto lay_out = [&](auto* out) {
    int ro0 = 0, rr0 = 0;                            // first positions of the two received runs
    if (live) {
      int pos = rp0 - base;
      for (int m = sr.hh_lo; m < sr.hh_lo + (int)sr.hh_n; ++m)
        if (m != i) out[pos++] = m;
      // the row's own draws: consecutive entries of the leaf's own range (the lanes
      // of a wave read one contiguous stretch of it)
      const uint32_t* own = ob + (wb + inc - c);
      for (int q = 0; q < ko; ++q) out[pos + q] = (int)col_word((uint32_t)((int)own[q] - dl), 1u);
      pos += ko;
      ro0 = pos;
      pos += co;
      for (int q = 0; q < kr; ++q) out[pos + q] = (int)col_word((uint32_t)((int)own[ko + q] - dl), 2u);
      pos += kr;
      rr0 = pos;
      cur[2 * tid] = ro0;
      cur[2 * tid + 1] = rr0;
    }
    __syncthreads();
    // received entries to the next position of their run
    auto put = [&](const uint2& v) {
      const int k = rkey(v.x);
      out[atomicAdd(&cur[k], 1)] = (int)col_word(v.y, (uint32_t)(k & 1) + 1u);
    };
#pragma unroll
    for (int j = 0; j < PB_ROWS_PER; ++j)
      if (j * NR + tid < nreg) put(x[j]);
    for (int e = lo + nreg + tid; e < hi; e += NR) put(d.pb_buf2[e]);
    __syncthreads();
    // each run sorted by initiator (the network bits are the same within a run)
    if (live) {
      const int runs[2][2] = {{ro0, ro0 + co}, {rr0, rr0 + cr}};
      for (int r = 0; r < 2; ++r) {
        const int a = runs[r][0], b = runs[r][1];
        for (int y0 = a + 1; y0 < b; ++y0) {
          const uint32_t v = (uint32_t)out[y0];
          int y = y0 - 1;
          while (y >= a && (uint32_t)out[y] > v) {
            out[y + 1] = out[y];
            --y;
          }
          out[y + 1] = (int)v;
        }
      }
    }
  };
  if (!staged) {
    lay_out(d.col + base);
    return;
  }
  lay_out(scol);
  __syncthreads();
  // the staged range leaves in 16-byte stores between its first and last 16-byte
  // boundaries in the column array (the array itself starts on one)
  const int n = end - base, head = min(n, (4 - (base & 3)) & 3), nv = (n - head) >> 2;
  if (tid < head) d.col[base + tid] = scol[tid];
  for (int v = tid; v < nv; v += NR) {
    const int k = head + 4 * v;
    *reinterpret_cast<int4*>(d.col + base + k) = make_int4(scol[k], scol[k + 1], scol[k + 2], scol[k + 3]);
  }
  for (int k = head + 4 * nv + tid; k < n; k += NR) d.col[base + k] = scol[k];
}

// Named steps of a day's graph build.  With the partitioned builder off (populations
// too large for 1024 level-1 digits) the claim-based builder of k_graph.hip runs.
int build_steps(const Dev& d) { return d.pb_on ? 7 : 5; }

const char* build_step_name(const Dev& d, int k) {
  static const char* pb[7] = {"pb_gen", "pb_scan1", "pb_scatter1", "pb_hist2",
                              "pb_scatter2", "pb_leaves", "pb_rows"};
  static const char* cl[5] = {"clear", "count", "scan", "fill", "canon"};
  return d.pb_on ? pb[k] : cl[k];
}

static size_t gen_lds(const Dev& d) {
  return ((size_t)d.pb_bcap + (size_t)d.pb_bpw * ((d.pb_nb1 + 1) / 2)) * 4;
}
static size_t rows_lds(const Dev& d) { return (size_t)d.pb_asm_cap * 4; }

hipError_t prepare_build(const Dev& d) {
  if (!d.pb_on) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_pb_rows<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)rows_lds(d));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pb_rows<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)rows_lds(d));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pb_gen, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)gen_lds(d));
}

void launch_build_step(const Dev& d, int k, hipStream_t s) {
  if (!d.pb_on) {
    switch (k) {
      case 0: launch_clear_recv(d, s); break;
      case 1: launch_count(d, s); break;
      case 2: launch_scan(d, s); break;
      case 3: launch_fill(d, s); break;
      default: launch_canon(d, s); break;
    }
    return;
  }
  switch (k) {
    case 0: hipLaunchKernelGGL(k_pb_gen, dim3(d.pb_ngrid), dim3(PB_THREADS), gen_lds(d), s, d); break;
    case 1:
      if ((int64_t)d.pb_nb1 * d.pb_nbatch <= 1024 * PB_S1_ONE) {
        hipLaunchKernelGGL(k_pb_s1_one, dim3(1), dim3(1024), 0, s, d);
        break;
      }
      hipLaunchKernelGGL(k_pb_s1a, dim3(d.pb_s1_nparts), dim3(TILE), 0, s, d);
      hipLaunchKernelGGL(k_pb_parts, dim3(1), dim3(1024), 0, s, d.pb_part, d.pb_s1_nparts);
      hipLaunchKernelGGL(k_pb_s1c, dim3(d.pb_s1_nparts), dim3(TILE), 0, s, d);
      hipLaunchKernelGGL(k_pb_buckets, dim3(1), dim3(1024), 0, s, d);
      break;
    case 2: hipLaunchKernelGGL(k_pb_scatter1, dim3(d.pb_ngrid), dim3(PB_THREADS), 0, s, d); break;
    case 3:
      hipLaunchKernelGGL(k_pb_hist2, dim3(d.pb_maxch), dim3(TILE), 0, s, d);
      hipLaunchKernelGGL(k_pb_s2, dim3(d.pb_nb1), dim3(PB_S2_SCAN), 0, s, d);
      break;
    case 4: hipLaunchKernelGGL(k_pb_scatter2, dim3(d.pb_maxch), dim3(PB_S2_THREADS), 0, s, d); break;
    case 5:                                  // one group of leaves: the row pass sums
      if (d.pb_ntgrp > 1) {
        hipLaunchKernelGGL(k_pb_tsum, dim3(d.pb_ntgrp), dim3(PB_TGRP), 0, s, d);
        hipLaunchKernelGGL(k_pb_parts, dim3(1), dim3(1024), 0, s, d.pb_tpart, d.pb_ntgrp);
      }
      break;
    default:
      if (d.pb_lb == 9)
        hipLaunchKernelGGL(k_pb_rows<2>, dim3(d.pb_nlv), dim3(2 * TILE), rows_lds(d), s, d);
      else
        hipLaunchKernelGGL(k_pb_rows<1>, dim3(d.pb_nlv), dim3(TILE), rows_lds(d), s, d);
      break;
  }
}

}  // namespace abm
