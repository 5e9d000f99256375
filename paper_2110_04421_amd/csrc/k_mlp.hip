// Calibration network 192 -> 256 -> 256 -> 16 on the matrix cores: BF16 operands,
// FP32 accumulation (v_mfma_f32_16x16x32_bf16), FP32 master weights with Adam.
//
// One GEMM kernel serves every layer and every gradient: C[M,N] = A[M,K] B[K,N] with
// operands read through arbitrary (row, column) strides from FP32 or BF16 memory,
// rounded to BF16 (nearest, ties to even) when staged in LDS, plus an epilogue (bias,
// ReLU, mask by a ReLU output, FP32 and/or BF16 stores).  A 64x64 output tile per
// workgroup, 4 waves of 32x32 (2x2 MFMA blocks of 16x16), K in steps of 32.
#include <mutex>
#include <unordered_map>

#include "abm_internal.h"

namespace abm {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int GT = 64;   // output tile
constexpr int GK = 32;   // K step

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t load_bf16(const float* p, int64_t o) { return to_bf16(p[o]); }
__device__ __forceinline__ uint16_t load_bf16(const uint16_t* p, int64_t o) { return p[o]; }

// Eight consecutive elements p[o .. o + 8) (o a multiple of 8) as BF16, or zeros.
__device__ __forceinline__ uint4 load8(const uint16_t* p, int64_t o, bool ok) {
  return ok ? *reinterpret_cast<const uint4*>(p + o) : make_uint4(0u, 0u, 0u, 0u);
}
__device__ __forceinline__ uint4 load8(const float* p, int64_t o, bool ok) {
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
  if (ok) {
    a = *reinterpret_cast<const float4*>(p + o);
    b = *reinterpret_cast<const float4*>(p + o + 4);
  }
  return make_uint4((uint32_t)to_bf16(a.x) | ((uint32_t)to_bf16(a.y) << 16),
                    (uint32_t)to_bf16(a.z) | ((uint32_t)to_bf16(a.w) << 16),
                    (uint32_t)to_bf16(b.x) | ((uint32_t)to_bf16(b.y) << 16),
                    (uint32_t)to_bf16(b.z) | ((uint32_t)to_bf16(b.w) << 16));
}
// The eight values down a column of an LDS tile: dst[q * GK] = value q.
__device__ __forceinline__ void store_col(uint16_t* dst, const uint4& v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dst[(2 * q) * GK] = (uint16_t)(w[q] & 0xFFFFu);
    dst[(2 * q + 1) * GK] = (uint16_t)(w[q] >> 16);
  }
}

struct Gemm {
  int M, N, K;
  int64_t sam, sak;          // A(m, k) = A[m * sam + k * sak]
  int64_t sbn, sbk;          // B(k, n) = B[n * sbn + k * sbk]
  const uint16_t* bias;      // bf16 [N] or null
  const float* biasf;        // fp32 [N] or null
  int relu;
  const uint16_t* mask;      // bf16 [M][N] (row stride N): multiply by (mask > 0)
  float* C;                  // fp32 out [M][N] (row stride N) or null
  uint16_t* Cb;              // bf16 out [M][N] or null
  int avec, bvec;            // staging form of A, B: 1 rows contiguous in k, 2 contiguous
                             // along the rows, 0 element by element (set by gemm())
};

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm(Gemm g, const TA* A, const TB* B) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GT][GK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GK];   // Bs[n][k]
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging: thread -> (row r = tid / 4, k chunk c = (tid % 4) * 8).  An operand whose
  // rows are contiguous in k (vec 1) is loaded 8 elements at a time along a row; one
  // contiguous along the rows (vec 2: 8 rows of one k) is loaded 8 rows at a time with
  // thread -> (k = tid / 8, row chunk (tid % 8) * 8) and stored down the tile's column.
  const int sr = threadIdx.x >> 2, sc = (threadIdx.x & 3) * 8;
  const int tk = threadIdx.x >> 3, tc = (threadIdx.x & 7) * 8;
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    {
      if (g.avec == 1) {
        const int m = m0 + sr, k = k0 + sc;
        *reinterpret_cast<uint4*>(&As[sr][sc]) = load8(A, (int64_t)m * g.sam + k, m < g.M && k < g.K);
      } else if (g.avec == 2) {
        const int m = m0 + tc, k = k0 + tk;
        store_col(&As[tc][tk], load8(A, (int64_t)m + (int64_t)k * g.sak, m < g.M && k < g.K));
      } else {
        const int m = m0 + sr, k = k0 + sc;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          As[sr][sc + q] = (m < g.M && k + q < g.K) ? load_bf16(A, (int64_t)m * g.sam + (int64_t)(k + q) * g.sak)
                                                     : (uint16_t)0;
      }
      if (g.bvec == 1) {
        const int n = n0 + sr, k = k0 + sc;
        *reinterpret_cast<uint4*>(&Bs[sr][sc]) = load8(B, (int64_t)n * g.sbn + k, n < g.N && k < g.K);
      } else if (g.bvec == 2) {
        const int n = n0 + tc, k = k0 + tk;
        store_col(&Bs[tc][tk], load8(B, (int64_t)n + (int64_t)k * g.sbk, n < g.N && k < g.K));
      } else {
        const int n = n0 + sr, k = k0 + sc;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          Bs[sr][sc + q] = (n < g.N && k + q < g.K) ? load_bf16(B, (int64_t)n * g.sbn + (int64_t)(k + q) * g.sbk)
                                                     : (uint16_t)0;
      }
    }
    __syncthreads();
    const int r = lane & 15, kc = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      __builtin_memcpy(&a[i], &As[wm + 16 * i + r][kc], 16);
      __builtin_memcpy(&b[i], &Bs[wn + 16 * i + r][kc], 16);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // accumulator layout: lane holds column (lane % 16), rows 4 * (lane / 16) + 0..3
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][q];
        if (g.bias) v += from_bf16(g.bias[n]);
        if (g.biasf) v += g.biasf[n];
        if (g.relu) v = fmaxf(v, 0.f);
        if (g.mask && !(from_bf16(g.mask[(int64_t)m * g.N + n]) > 0.f)) v = 0.f;
        if (g.C) g.C[(int64_t)m * g.N + n] = v;
        if (g.Cb) g.Cb[(int64_t)m * g.N + n] = to_bf16(v);
      }
}

template <typename TA, typename TB>
void gemm(const Gemm& g0, const TA* A, const TB* B, hipStream_t s) {
  Gemm g = g0;
  const auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
  g.avec = !al(A) ? 0 : (g.sak == 1 && g.sam % 8 == 0 && g.K % 8 == 0) ? 1
           : (g.sam == 1 && g.sak % 8 == 0 && g.M % 8 == 0) ? 2 : 0;
  g.bvec = !al(B) ? 0 : (g.sbk == 1 && g.sbn % 8 == 0 && g.K % 8 == 0) ? 1
           : (g.sbn == 1 && g.sbk % 8 == 0 && g.N % 8 == 0) ? 2 : 0;
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT);
  hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(256), 0, s, g, A, B);
}

__global__ void k_to_bf16(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// y = x, and the batch size recorded in the workspace header (one lane)
__global__ void k_copy_f32(const float* x, float* y, int64_t n, int32_t* hdr, int32_t B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
  if (i == 0) *hdr = B;
}

// Column sums of an FP32 [rows][cols] matrix, rows in order.
// Column sums (bias gradients): a workgroup takes 64 columns; wave w adds rows w,
// w + 4, ... of its lane's column (each load a coalesced 256-byte row piece), and the
// four wave sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float* x, int rows, int cols, float* out) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (c < cols)
    for (int r = wv; r < rows; r += 4) s += x[(int64_t)r * cols + c];
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && c < cols) out[c] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// dY = 2 (y - t) / (B n_out) on the first n_out outputs, 0 elsewhere; loss = mean
// squared error (one workgroup, fixed-order reduction).
__global__ __launch_bounds__(256) void k_mse(const float* y, const float* t, int B, int n_out, float* dy,
                                             float* loss) {
  __shared__ float red[256];
  const int n = B * ABM_MLP_OUT;
  const float scale = 2.f / (float)(B * n_out);
  float acc = 0.f;
  for (int k = threadIdx.x; k < n; k += 256) {
    const int o = k % ABM_MLP_OUT;
    float diff = 0.f;
    if (o < n_out) diff = y[k] - t[(int64_t)(k / ABM_MLP_OUT) * ABM_MLP_OUT + o];
    dy[k] = scale * diff;
    acc += diff * diff;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)(B * n_out);
}

__global__ void k_adam(float* w, uint16_t* wb, float* m, float* v, const float* g, float lr, float b1,
                       float b2, float eps, float c1, float c2, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = to_bf16(wi);
}

// Parameter blob offsets (elements).
constexpr int64_t OW1 = 0, OB1 = OW1 + 256 * 192, OW2 = OB1 + 256, OB2 = OW2 + 256 * 256,
                  OW3 = OB2 + 256, OB3 = OW3 + 16 * 256;

// Workspace for a batch of B: [hdr 256 B][Xb bf16 B*192][H1 bf16 B*256][H2 bf16 B*256]
// [Y f32 B*16][dY f32 B*16][dH2 f32 B*256][dH1 f32 B*256].
struct MlpWs {
  int32_t* hdr;
  uint16_t *xb, *h1, *h2;
  float *y, *dy, *dh2, *dh1;
  size_t total;
};

constexpr size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Bytes of the layout below for a batch of B (the sum mlp_layout takes).
constexpr size_t mlp_ws_bytes(int64_t B) {
  size_t o = 256;
  o = al(o + (size_t)B * 192 * 2);
  o = al(o + (size_t)B * 256 * 2);
  o = al(o + (size_t)B * 256 * 2);
  o = al(o + (size_t)B * 16 * 4);
  o = al(o + (size_t)B * 16 * 4);
  o = al(o + (size_t)B * 256 * 4);
  o = al(o + (size_t)B * 256 * 4);
  return o;
}
// The forward pass touches only the layout's first five parts (header, Xb, H1, H2, Y).
constexpr size_t mlp_fwd_bytes(int64_t B) {
  size_t o = 256;
  o = al(o + (size_t)B * 192 * 2);
  o = al(o + (size_t)B * 256 * 2);
  o = al(o + (size_t)B * 256 * 2);
  o = al(o + (size_t)B * 16 * 4);
  return o;
}

MlpWs mlp_layout(void* base, int64_t B) {
  MlpWs w{};
  char* p = (char*)base;
  size_t o = 256;
  auto take = [&](size_t bytes) {
    char* q = p + o;
    o = al(o + bytes);
    return q;
  };
  w.hdr = (int32_t*)p;
  w.xb = (uint16_t*)take(B * 192 * 2);
  w.h1 = (uint16_t*)take(B * 256 * 2);
  w.h2 = (uint16_t*)take(B * 256 * 2);
  w.y = (float*)take(B * 16 * 4);
  w.dy = (float*)take(B * 16 * 4);
  w.dh2 = (float*)take(B * 256 * 4);
  w.dh1 = (float*)take(B * 256 * 4);
  w.total = o;
  return w;
}

Gemm plain(int M, int N, int K) {
  Gemm g{};
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace abm

using namespace abm;

// The batch of the last forward enqueued on each workspace, kept on the host so that
// the backward checks it without waiting for the stream.
namespace {
std::mutex batch_mu;
std::unordered_map<const void*, int32_t> batch_of;
void remember_batch(const void* ws, int32_t B) {
  std::lock_guard<std::mutex> g(batch_mu);
  batch_of[ws] = B;
}
int32_t last_batch(const void* ws) {
  std::lock_guard<std::mutex> g(batch_mu);
  const auto it = batch_of.find(ws);
  return it == batch_of.end() ? -1 : it->second;
}
// The forward pass on workspace w: inputs rounded to BF16, two hidden layers with bias
// and ReLU, the output layer in FP32, copied to y.
hipError_t enqueue_forward(const MlpWs& w, const uint16_t* P, const float* d_x, int32_t B, float* d_y,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks((int64_t)B * 192)), dim3(256), 0, s, d_x, w.xb, (int64_t)B * 192);
  Gemm g = plain(B, 256, 192);
  g.sam = 192; g.sak = 1; g.sbn = 192; g.sbk = 1;
  g.bias = P + OB1; g.relu = 1; g.Cb = w.h1;
  gemm(g, (const uint16_t*)w.xb, P + OW1, s);
  g = plain(B, 256, 256);
  g.sam = 256; g.sak = 1; g.sbn = 256; g.sbk = 1;
  g.bias = P + OB2; g.relu = 1; g.Cb = w.h2;
  gemm(g, (const uint16_t*)w.h1, P + OW2, s);
  g = plain(B, 16, 256);
  g.sam = 256; g.sak = 1; g.sbn = 256; g.sbk = 1;
  g.bias = P + OB3; g.C = w.y;
  gemm(g, (const uint16_t*)w.h2, P + OW3, s);
  hipLaunchKernelGGL(k_copy_f32, dim3(blocks((int64_t)B * 16)), dim3(256), 0, s, (const float*)w.y, d_y,
                     (int64_t)B * 16, w.hdr, B);
  return hipGetLastError();
}

// Scratch of the allocation-free forward: the activations of one batch of at most
// ABM_MLP_NOALLOC_MAX_BATCH rows, in the layout of mlp_layout (about 1.5 MB).  Each
// GPU holds its own copy for the life of the process.  Its device address is taken
// once per device (with that device current) and kept; the array's name is a host-side
// stand-in and is never handed to a kernel.
constexpr size_t NOALLOC_BYTES = mlp_fwd_bytes(ABM_MLP_NOALLOC_MAX_BATCH);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

hipError_t scratch_base(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int abm_mlp_workspace_size(int32_t max_batch, size_t* bytes) {
  if (!bytes || max_batch < 1) return ABM_E_ARG;
  *bytes = mlp_ws_bytes(max_batch);
  return ABM_OK;
}

int abm_mlp_forward(void* d_ws, size_t ws_bytes, const uint16_t* P, const float* d_x, int32_t B,
                    float* d_y, void* stream) {
  if (!d_ws || !P || !d_x || !d_y || B < 1) return ABM_E_ARG;
  MlpWs w = mlp_layout(d_ws, B);
  if (w.total > ws_bytes) return ABM_E_WORKSPACE;
  if (enqueue_forward(w, P, d_x, B, d_y, (hipStream_t)stream) != hipSuccess) return ABM_E_HIP;
  remember_batch(d_ws, B);
  return ABM_OK;
}

int abm_mlp_forward_noalloc(const uint16_t* P, const float* d_x, int32_t B, float* d_y, void* stream) {
  if (!P || !d_x || !d_y || B < 1) return ABM_E_ARG;
  if (B > ABM_MLP_NOALLOC_MAX_BATCH) return ABM_E_WORKSPACE;
  void* base = nullptr;
  if (scratch_base(&base) != hipSuccess) return ABM_E_HIP;
  MlpWs w = mlp_layout(base, B);
  if (enqueue_forward(w, P, d_x, B, d_y, (hipStream_t)stream) != hipSuccess) return ABM_E_HIP;
  return ABM_OK;
}

int abm_mlp_backward(void* d_ws, size_t ws_bytes, const uint16_t* P, const float* d_target, int32_t B,
                     int32_t n_out, float* G, float* d_loss, void* stream) {
  if (!d_ws || !P || !d_target || !G || B < 1 || n_out < 1 || n_out > ABM_MLP_OUT) return ABM_E_ARG;
  MlpWs w = mlp_layout(d_ws, B);
  if (w.total > ws_bytes) return ABM_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (last_batch(d_ws) != B) return ABM_E_STATE;     // the last forward used another batch
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, (const float*)w.y, d_target, B, n_out, w.dy, d_loss);
  // dW3 = dY^T H2 ; db3 = colsum dY
  Gemm g = plain(16, 256, B);
  g.sam = 1; g.sak = 16; g.sbn = 1; g.sbk = 256; g.C = G + OW3;
  gemm(g, (const float*)w.dy, (const uint16_t*)w.h2, s);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, (const float*)w.dy, B, 16, G + OB3);
  // dH2 = (dY W3) * [H2 > 0]
  g = plain(B, 256, 16);
  g.sam = 16; g.sak = 1; g.sbn = 1; g.sbk = 256; g.mask = w.h2; g.C = w.dh2;
  gemm(g, (const float*)w.dy, P + OW3, s);
  // dW2 = dH2^T H1 ; db2
  g = plain(256, 256, B);
  g.sam = 1; g.sak = 256; g.sbn = 1; g.sbk = 256; g.C = G + OW2;
  gemm(g, (const float*)w.dh2, (const uint16_t*)w.h1, s);
  hipLaunchKernelGGL(k_colsum, dim3(4), dim3(256), 0, s, (const float*)w.dh2, B, 256, G + OB2);
  // dH1 = (dH2 W2) * [H1 > 0]
  g = plain(B, 256, 256);
  g.sam = 256; g.sak = 1; g.sbn = 1; g.sbk = 256; g.mask = w.h1; g.C = w.dh1;
  gemm(g, (const float*)w.dh2, P + OW2, s);
  // dW1 = dH1^T Xb ; db1
  g = plain(256, 192, B);
  g.sam = 1; g.sak = 256; g.sbn = 1; g.sbk = 192; g.C = G + OW1;
  gemm(g, (const float*)w.dh1, (const uint16_t*)w.xb, s);
  hipLaunchKernelGGL(k_colsum, dim3(4), dim3(256), 0, s, (const float*)w.dh1, B, 256, G + OB1);
  return hipGetLastError() == hipSuccess ? ABM_OK : ABM_E_HIP;
}

int abm_mlp_adam(float* d_master, uint16_t* d_params, float* d_m, float* d_v, const float* d_grads,
                 float lr, float b1, float b2, float eps, int32_t step, void* stream) {
  if (!d_master || !d_params || !d_m || !d_v || !d_grads || step < 1) return ABM_E_ARG;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(ABM_MLP_NPARAM)), dim3(256), 0, (hipStream_t)stream, d_master,
                     d_params, d_m, d_v, d_grads, lr, b1, b2, eps, c1, c2, (int64_t)ABM_MLP_NPARAM);
  return hipGetLastError() == hipSuccess ? ABM_OK : ABM_E_HIP;
}

}  // extern "C"
