// Relaxed (differentiable) day step and its hand-written adjoint.
//
// Forward, per day t and agent j (eqs. 1-2 with the hard draw u < p replaced by a
// Gumbel-softmax sample on the same uniform u):
//   inf_i   = sum_{tau=1..L} Atab[tau] e_i(t - tau)                 (k_soft_inf)
//   sigma_j = sum_{e in row j} w_e inf_src(e)                        (k_soft_message)
//   lambda  = coef[a_j] sigma_j,  y = sigmoid((log expm1(lambda dt) - logit u) / tau_g)
//   e_j(t)  = s_j y_j,  s_j <- s_j - e_j,  c_r(t) = sum_{j in r} e_j  (k_soft_update)
// Reverse, per day t from the last one (checkpoints every `seg` days, the segment
// recomputed forward with sigma, y, s kept, the day's graph rebuilt from Philox):
//   ebar    = dL/dc(t) + sum_tau Atab[tau] infbar_j(t + tau) - sbar_j(t + 1)
//   sbar(t) = sbar(t + 1) + ebar y,   ybar = ebar s
//   lbar    = ybar y (1 - y) / tau_g * dt / p  (0 where lambda = 0)
//   infbar_i(t) = sum_{e in row i} w_e coef_src lbar_src   (same CSR: the graph is symmetric)
//   dR += lbar kappa S[a] sigma,  dS_a += lbar R kappa sigma.
// All reductions use fixed orders, so results are bitwise reproducible.
#include "abm_internal.h"

namespace abm {

__device__ __forceinline__ int ring(int t) { return ((t % WIN) + WIN) % WIN; }

__device__ __forceinline__ float sigmoidf(float z) {
  const float e = __expf(-fabsf(z));
  return z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}

// Fixed-order sum over the workgroup (4 waves); result valid in thread 0.
__device__ __forceinline__ float block_sum(float v, float* lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int q = 0; q < TILE / 64; ++q) s += lds[q];
  return s;
}

__global__ __launch_bounds__(TILE) void k_soft_zero(Dev d) {
  const int64_t n = (int64_t)WIN * d.N;
  for (int64_t k = (int64_t)blockIdx.x * TILE + threadIdx.x; k < n; k += (int64_t)gridDim.x * TILE) {
    d.ehist[k] = 0.f;
    d.ibar[k] = 0.f;
  }
  for (int64_t k = (int64_t)blockIdx.x * TILE + threadIdx.x; k < d.N; k += (int64_t)gridDim.x * TILE) {
    d.s[k] = 1.f;
    d.s_bar[k] = 0.f;
  }
}

__global__ void k_soft_seed(Dev d, const int32_t* seeds, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = seeds[k];
  d.s[i] = 0.f;
  d.ehist[(size_t)ring(-1) * d.N + i] = 1.f;     // exposed on day -1
}

__global__ __launch_bounds__(TILE) void k_soft_inf(Dev d) {
  const int i = blockIdx.x * TILE + threadIdx.x;
  if (i >= d.N) return;
  const int t = *d.day;
  float acc = 0.f;
  for (int tau = 1; tau <= d.e_days + d.i_days; ++tau)
    acc += d.atab[tau] * d.ehist[(size_t)ring(t - tau) * d.N + i];
  d.inf[i] = acc;
}

// out_j = sum_{e in row j} w_e x[src_e]: the tile's edge range is staged through LDS in
// chunks; each lane then sums its own row left to right (same order as the forward).
__global__ __launch_bounds__(TILE) void k_soft_message(Dev d, const float* x, float* out) {
  __shared__ float term[MSG_CHUNK];
  if (*d.flags) return;
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const bool live = i < tl.z;
  const int e0 = d.row_ptr[tl.y], e1 = d.row_ptr[tl.z];
  const int rs = live ? d.row_ptr[i] : 0, re = live ? d.row_ptr[i + 1] : 0;
  float sum = 0.f;
  for (int c0 = e0; c0 < e1; c0 += MSG_CHUNK) {
    const int cn = min(MSG_CHUNK, e1 - c0);
    for (int k = threadIdx.x; k < cn; k += TILE) {
      const int e = c0 + k;
      const uint32_t c = (uint32_t)d.col[e];
      const uint32_t src = (c & COL_AGENT) < (uint32_t)d.N ? (c & COL_AGENT) : 0u;
      term[k] = col_weight(c, d.w_h, d.w_o, d.w_r) * x[src];
    }
    __syncthreads();
    const int lo = max(rs, c0), hi = min(re, c0 + cn);
    for (int e = lo; e < hi; ++e) sum += term[e - c0];
    __syncthreads();
  }
  if (live) out[i] = sum;
}

__device__ __forceinline__ float logit_u(const Dev& d, const RepInfo& ri, int i, int t) {
  const uint4 b = philox((uint32_t)(i - ri.start), (uint32_t)t, ri.stream, P_AGENT << 24, d.key0, d.key1);
  const float u = u01(b.x);
  return logf(u) - log1pf(-u);
}

__global__ __launch_bounds__(TILE) void k_soft_update(Dev d, int32_t seg_slot) {
  __shared__ float lds[TILE / 64];
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const bool live = i < tl.z;
  const int t = *d.day;
  float e = 0.f;
  if (live) {
    const RepInfo& ri = d.rep[tl.x];
    const float sigma = d.sigma[i];
    const float lam = ri.coef[d.age[i]] * sigma;
    const float x = lam * d.dt;
    float y = 0.f;                       // the sample the state takes
    if (x > 0.f) {
      if (d.straight) {
        // the hard step's draw: u < 1 - exp(-lambda dt) in FP64 on the same uniform
        const uint4 b = philox((uint32_t)(i - ri.start), (uint32_t)t, ri.stream, P_AGENT << 24, d.key0, d.key1);
        const double p = -expm1(-(double)lam * (double)d.dt);
        y = (double)u01(b.x) < p ? 1.f : 0.f;
      } else {
        y = sigmoidf((logf(expm1f(x)) - logit_u(d, ri, i, t)) / d.gtau);
      }
    }
    const float s = d.s[i];
    e = s * y;
    if (seg_slot >= 0) {
      const size_t o = (size_t)seg_slot * d.N + i;
      d.seg_sigma[o] = sigma;
      d.seg_y[o] = y;
      d.seg_s[o] = s;
    }
    d.s[i] = s - e;
    d.ehist[(size_t)ring(t) * d.N + i] = e;
  }
  const float tot = block_sum(e, lds);
  if (threadIdx.x == 0) d.gpart[(size_t)blockIdx.x * ABM_N_THETA] = tot;
}

// Daily relaxed incidence per replicate: its tiles' partial sums in tile order.
// Per replicate, the sums of its tiles' partials in slots [0, NQ): lane l adds tiles l,
// l + 256, ... in order, then the lanes are added in a fixed tree (the order, and so
// the rounding, depends only on the replicate's tile count).  out[q] on lane 0.
template <int NQ>
__device__ __forceinline__ void rep_sums(const Dev& d, const RepInfo& ri, float (*red)[NQ], float* out) {
  float acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.f;
  for (int m = threadIdx.x; m < ri.ntiles; m += TILE) {
    const float* g = d.gpart + (size_t)(ri.tile0 + m) * ABM_N_THETA;
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += g[q];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o);
    if (lane == 0) red[wv][q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// One workgroup per replicate; the last to finish advances the day (every workgroup
// has read it by then).
__global__ __launch_bounds__(TILE) void k_soft_finalize(Dev d) {
  __shared__ float red[TILE / 64][1];
  const int r = blockIdx.x;
  const int t = *d.day;
  float c;
  rep_sums<1>(d, d.rep[r], red, &c);
  if (threadIdx.x == 0) {
    if (t < d.T) d.soft_inc[(size_t)r * d.T + t] = c;
    if (atomicAdd(d.fin_done, 1) == (int)gridDim.x - 1) {
      *d.fin_done = 0;
      *d.day = t + 1;
    }
  }
}

// Checkpoint slot k = susceptible mass + the exposure ring.
__global__ __launch_bounds__(TILE) void k_soft_ckpt(Dev d, int32_t k, int32_t load) {
  const int64_t n = (int64_t)(WIN + 1) * d.N;
  float* ck = d.ckpt + (size_t)k * n;
  for (int64_t q = (int64_t)blockIdx.x * TILE + threadIdx.x; q < n; q += (int64_t)gridDim.x * TILE) {
    float* live = q < d.N ? d.s + q : d.ehist + (q - d.N);
    if (load) *live = ck[q];
    else ck[q] = *live;
  }
}

__global__ __launch_bounds__(TILE) void k_adj_zero(Dev d) {
  const int64_t n = (int64_t)WIN * d.N;
  for (int64_t k = (int64_t)blockIdx.x * TILE + threadIdx.x; k < n; k += (int64_t)gridDim.x * TILE)
    d.ibar[k] = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * TILE + threadIdx.x; k < d.N; k += (int64_t)gridDim.x * TILE)
    d.s_bar[k] = 0.f;
  for (int k = blockIdx.x * TILE + threadIdx.x; k < d.R * ABM_N_THETA; k += gridDim.x * TILE)
    d.gtheta[k] = 0.f;
}

__global__ __launch_bounds__(TILE) void k_adj_day(Dev d, int32_t t, int32_t seg_slot) {
  __shared__ float lds[TILE / 64];
  const int4 tl = d.tiles[blockIdx.x];
  const int i = tl.y + threadIdx.x;
  const bool live = i < tl.z;
  const RepInfo& ri = d.rep[tl.x];
  float gR = 0.f, gS[ABM_N_AGE];
#pragma unroll
  for (int a = 0; a < ABM_N_AGE; ++a) gS[a] = 0.f;
  if (live) {
    const size_t o = (size_t)seg_slot * d.N + i;
    const float y = d.seg_y[o], s = d.seg_s[o], sigma = d.seg_sigma[o];
    float acc = 0.f;
    for (int tau = 1; tau <= d.e_days + d.i_days; ++tau)
      acc += d.atab[tau] * d.ibar[(size_t)ring(t + tau) * d.N + i];
    const float ebar = d.dL[(size_t)tl.x * d.T + t] + acc - d.s_bar[i];
    d.s_bar[i] = d.s_bar[i] + ebar * y;
    const float ybar = ebar * s;
    const int a = d.age[i];
    const float lam = ri.coef[a] * sigma;
    const float x = lam * d.dt;
    float lbar = 0.f;
    if (x > 0.f) {
      const float p = -expm1f(-x);
      // straight-through: the saved sample is the hard one; the derivative is the
      // relaxed sample's, recomputed from the same uniform
      const float ys = d.straight ? sigmoidf((logf(expm1f(x)) - logit_u(d, ri, i, t)) / d.gtau) : y;
      lbar = ybar * ys * (1.f - ys) / d.gtau * d.dt / p;
    }
    d.vtmp[i] = ri.coef[a] * lbar;
    gR = lbar * (d.kappa * ri.S[a]) * sigma;
#pragma unroll
    for (int q = 0; q < ABM_N_AGE; ++q) gS[q] = (q == a) ? lbar * ri.rk * sigma : 0.f;
  }
  float v = block_sum(gR, lds);
  if (threadIdx.x == 0) d.gpart[(size_t)blockIdx.x * ABM_N_THETA] = v;
#pragma unroll
  for (int q = 0; q < ABM_N_AGE; ++q) {
    v = block_sum(gS[q], lds);
    if (threadIdx.x == 0) d.gpart[(size_t)blockIdx.x * ABM_N_THETA + 1 + q] = v;
  }
}

// One workgroup per replicate: the day's gradient partials of its tiles, added to dθ.
__global__ __launch_bounds__(TILE) void k_adj_theta(Dev d) {
  __shared__ float red[TILE / 64][ABM_N_THETA];
  const int r = blockIdx.x;
  float g[ABM_N_THETA];
  rep_sums<ABM_N_THETA>(d, d.rep[r], red, g);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < ABM_N_THETA; ++q) d.gtheta[(size_t)r * ABM_N_THETA + q] += g[q];
}

static unsigned grid_for(int64_t n) {
  const int64_t b = (n + TILE - 1) / TILE;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

void launch_soft_init(const Dev& d, const int32_t* seeds, int64_t nseeds, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_zero, dim3(grid_for((int64_t)WIN * d.N)), dim3(TILE), 0, s, d);
  if (nseeds > 0)
    hipLaunchKernelGGL(k_soft_seed, dim3((unsigned)((nseeds + 255) / 256)), dim3(256), 0, s, d, seeds, nseeds);
}
void launch_soft_inf(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_inf, dim3((d.N + TILE - 1) / TILE), dim3(TILE), 0, s, d);
}
void launch_soft_message(const Dev& d, const float* x, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_message, dim3(d.ntiles), dim3(TILE), 0, s, d, x, out);
}
void launch_soft_update(const Dev& d, int32_t seg_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_update, dim3(d.ntiles), dim3(TILE), 0, s, d, seg_slot);
}
void launch_soft_finalize(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_finalize, dim3(d.R), dim3(TILE), 0, s, d);
}
void launch_soft_ckpt_save(const Dev& d, int32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_ckpt, dim3(grid_for((int64_t)(WIN + 1) * d.N)), dim3(TILE), 0, s, d, k, 0);
}
void launch_soft_ckpt_load(const Dev& d, int32_t k, int32_t day, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_ckpt, dim3(grid_for((int64_t)(WIN + 1) * d.N)), dim3(TILE), 0, s, d, k, 1);
  launch_set_day(d, day, s);
}
void launch_adj_zero(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_zero, dim3(grid_for((int64_t)WIN * d.N)), dim3(TILE), 0, s, d);
}
void launch_adj_day(const Dev& d, int32_t t, int32_t seg_slot, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_day, dim3(d.ntiles), dim3(TILE), 0, s, d, t, seg_slot);
}
void launch_adj_theta(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_theta, dim3(d.R), dim3(TILE), 0, s, d);
}
void launch_adj_ibar(const Dev& d, int32_t t, hipStream_t s) {
  const int slot = ((t % WIN) + WIN) % WIN;
  launch_soft_message(d, d.vtmp, d.ibar + (size_t)slot * d.N, s);
}

}  // namespace abm
