// Small dense network (3 layers) on the gfx950 matrix cores: BF16 operands, FP32 accumulation.
// See include/gigaqbx_mlp.h for the contract. All matrix products go through one kernel built on
// v_mfma_f32_16x16x16bf16_1k (one wavefront per 16x16 output tile); biases, activations, the
// loss and Adam run in FP32 elementwise kernels. Reductions are fixed-order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gigaqbx_mlp.h"

typedef short gq_s4 __attribute__((ext_vector_type(4)));
typedef float gq_mf4 __attribute__((ext_vector_type(4)));

namespace {

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] (FP32, ldc) = op(A)[M x K] op(B)[K x N], BF16 operands.
// op(A)(i, k) = ta ? A[k lda + i] : A[i lda + k];  op(B)(k, j) = tb ? B[j ldb + k] : B[k ldb + j].
// Operand layout of the 16x16x16 instruction: A[i][k] in lane i + 16 (k / 4), element k % 4;
// B[k][j] in lane j + 16 (k / 4), element k % 4; D[4 (l / 16) + v][l % 16] in element v of lane l.
__global__ void __launch_bounds__(64) k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A,
                                                  int lda, int ta, const uint16_t *__restrict__ B,
                                                  int ldb, int tb, float *__restrict__ C, int ldc) {
  const int l = threadIdx.x, g = l >> 4, c16 = l & 15;
  const int i = blockIdx.y * 16 + c16, j = blockIdx.x * 16 + c16;
  // split-K: work-group z covers K rows [k_lo, k_hi) and writes slab z of C (slab stride M ldc)
  const int ks = (K + gridDim.z - 1) / gridDim.z;
  const int k_lo = min(K, (int)blockIdx.z * ((ks + 15) / 16 * 16));
  const int k_hi = min(K, k_lo + (ks + 15) / 16 * 16);
  C += (int64_t)blockIdx.z * M * ldc;
  gq_mf4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
    gq_s4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + 4 * g + e;
      const bool kin = k < k_hi;
      a[e] = (short)((kin && i < M) ? (ta ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k]) : 0);
      b[e] = (short)((kin && j < N) ? (tb ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j]) : 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = blockIdx.y * 16 + 4 * g + v, col = blockIdx.x * 16 + c16;
    if (row < M && col < N) C[(int64_t)row * ldc + col] = acc[v];
  }
}

// out[t] = sum over z of part[z n_el + t], z ascending (fixed order)
__global__ void k_sum_slabs(int n_el, int n_slab, const float *__restrict__ part,
                            float *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_el) return;
  float s = 0.f;
  for (int z = 0; z < n_slab; ++z) s += part[(int64_t)z * n_el + t];
  out[t] = s;
}

// X (n x n_in, FP32) -> Xb (n x in_pad, BF16, zero padded)
__global__ void k_pack_input(int64_t n, int n_in, int in_pad, const float *__restrict__ x,
                             uint16_t *__restrict__ xb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * in_pad) return;
  const int64_t r = t / in_pad;
  const int c = (int)(t % in_pad);
  xb[t] = c < n_in ? bf16(x[r * n_in + c]) : 0;
}

// Z += b; H = bf16(relu(Z))      (Z: n x H, FP32)
__global__ void k_bias_relu(int64_t n, int H, float *__restrict__ Z, const float *__restrict__ b,
                            uint16_t *__restrict__ hb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * H) return;
  const float z = Z[t] + b[t % H];
  Z[t] = z;
  hb[t] = bf16(z > 0.f ? z : 0.f);
}

// y = Zy[:, :n_out] + b3
__global__ void k_output(int64_t n, int n_out, int out_pad, const float *__restrict__ zy,
                         const float *__restrict__ b, float *__restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_out) return;
  const int64_t r = t / n_out;
  const int c = (int)(t % n_out);
  y[t] = zy[r * out_pad + c] + b[c];
}

// e = y - t; loss partial += w e^2; dY = 2 w e / (n n_out) (FP32 and BF16, out_pad columns)
__global__ void __launch_bounds__(256) k_loss_grad(int64_t n, int n_out, int out_pad,
                                                   const float *__restrict__ y,
                                                   const float *__restrict__ t,
                                                   const float *__restrict__ w, float scale,
                                                   float *__restrict__ dy, uint16_t *__restrict__ dyb,
                                                   float *__restrict__ part) {
  __shared__ float red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (i < n * out_pad) {
    const int64_t r = i / out_pad;
    const int c = (int)(i % out_pad);
    float g = 0.f;
    if (c < n_out) {
      const float e = y[r * n_out + c] - t[r * n_out + c];
      const float ww = w ? w[r * n_out + c] : 1.f;
      s = ww * e * e;
      g = 2.f * ww * e * scale;
    }
    dy[i] = g;
    dyb[i] = bf16(g);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dZ = dH * (Z > 0)  (FP32 and BF16)
__global__ void k_relu_back(int64_t n, int H, const float *__restrict__ dh, const float *__restrict__ z,
                            float *__restrict__ dz, uint16_t *__restrict__ dzb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * H) return;
  const float g = z[t] > 0.f ? dh[t] : 0.f;
  dz[t] = g;
  dzb[t] = bf16(g);
}

// out[c] = sum_r A[r lda + c] for c < N: one work-group per column, fixed-order tree reduction
__global__ void __launch_bounds__(256) k_colsum(int64_t n, int lda, const float *__restrict__ A,
                                                float *__restrict__ out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += A[r * lda + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void k_adam(int64_t np, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const float gg = g[t];
  const float mm = 0.9f * m[t] + 0.1f * gg;
  const float vv = 0.999f * v[t] + 0.001f * gg * gg;
  m[t] = mm;
  v[t] = vv;
  p[t] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

// BF16 padded copies of the weight matrices: W (rows x cols FP32) -> Wb (rows_pad x cols_pad)
__global__ void k_weight_bf16(int rows, int cols, int rows_pad, int cols_pad,
                              const float *__restrict__ w, uint16_t *__restrict__ wb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows_pad * cols_pad) return;
  const int r = t / cols_pad, c = t % cols_pad;
  wb[t] = (r < rows && c < cols) ? bf16(w[r * cols + c]) : 0;
}

int pad16(int x) { return (x + 15) / 16 * 16; }
constexpr int kMaxSplit = 256;
inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

struct gq_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int n_in = 0, n_h = 0, n_out = 0, in_pad = 0, out_pad = 0;
  int64_t np = 0, step = 0;
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;
  uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
  // batch workspace
  int64_t cap = 0;
  uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *dZb = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Zy = nullptr, *dY = nullptr, *dH = nullptr, *dZ = nullptr,
        *Ytmp = nullptr, *part = nullptr, *Gpart = nullptr;
  std::vector<void *> ws;
  // offsets of the parameter blocks
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
};

namespace {

gq_status mfail(gq_mlp *net, gq_status st, const std::string &m) {
  if (net) net->err = m;
  return st;
}

#define GQ_MLP_HIP(net, call)                                                                 \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return mfail(net, GQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
gq_status dalloc(gq_mlp *net, T *&p, size_t n, std::vector<void *> &list) {
  void *q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
    return mfail(net, GQ_ENOMEM, "hipMalloc");
  list.push_back(q);
  p = static_cast<T *>(q);
  return GQ_OK;
}

gq_status ensure_batch(gq_mlp *net, int64_t n) {
  if (n <= net->cap) return GQ_OK;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  for (void *p : net->ws) (void)hipFree(p);
  net->ws.clear();
  const int64_t H = net->n_h;
  gq_status s = GQ_OK;
#define A(ptr, cnt) if (s == GQ_OK) s = dalloc(net, net->ptr, (size_t)(cnt), net->ws)
  A(Xb, n * net->in_pad); A(H1b, n * H); A(H2b, n * H); A(dYb, n * net->out_pad); A(dZb, n * H);
  A(Z1, n * H); A(Z2, n * H); A(Zy, n * net->out_pad); A(dY, n * net->out_pad); A(dH, n * H);
  A(dZ, n * H); A(Ytmp, n * net->n_out); A(part, (n * net->out_pad + 255) / 256);
  A(Gpart, (int64_t)kMaxSplit * std::max<int64_t>(H * H, (int64_t)std::max(net->in_pad, net->out_pad) * H));
#undef A
  if (s == GQ_OK) net->cap = n;
  return s;
}

void gemm(gq_mlp *net, int M, int N, int K, const uint16_t *A, int lda, int ta, const uint16_t *B,
          int ldb, int tb, float *C, int ldc) {
  hipLaunchKernelGGL(k_gemm_bf16, dim3((N + 15) / 16, (M + 15) / 16, 1), dim3(64), 0, net->stream,
                     M, N, K, A, lda, ta, B, ldb, tb, C, ldc);
}

// Weight gradient C (M x N, ldc = N) = op(A) op(B) with a long contraction over the batch rows:
// split over up to kMaxSplit work-groups along K, partial products summed in fixed order.
void gemm_splitk(gq_mlp *net, int M, int N, int K, const uint16_t *A, int lda, int ta,
                 const uint16_t *B, int ldb, int tb, float *C) {
  const int split = std::max(1, std::min(kMaxSplit, K / 2048));
  hipLaunchKernelGGL(k_gemm_bf16, dim3((N + 15) / 16, (M + 15) / 16, split), dim3(64), 0,
                     net->stream, M, N, K, A, lda, ta, B, ldb, tb, net->Gpart, N);
  hipLaunchKernelGGL(k_sum_slabs, dim3(blocks((int64_t)M * N)), dim3(256), 0, net->stream, M * N,
                     split, net->Gpart, C);
}


void refresh_bf16(gq_mlp *net) {
  const int H = net->n_h;
  hipLaunchKernelGGL(k_weight_bf16, dim3(blocks((int64_t)net->in_pad * H)), dim3(256), 0, net->stream,
                     net->n_in, H, net->in_pad, H, net->P + net->oW1, net->W1b);
  hipLaunchKernelGGL(k_weight_bf16, dim3(blocks((int64_t)H * H)), dim3(256), 0, net->stream, H, H, H,
                     H, net->P + net->oW2, net->W2b);
  hipLaunchKernelGGL(k_weight_bf16, dim3(blocks((int64_t)H * net->out_pad)), dim3(256), 0,
                     net->stream, H, net->n_out, H, net->out_pad, net->P + net->oW3, net->W3b);
}

void forward(gq_mlp *net, int64_t n, const float *x) {
  const int H = net->n_h;
  hipLaunchKernelGGL(k_pack_input, dim3(blocks(n * net->in_pad)), dim3(256), 0, net->stream, n,
                     net->n_in, net->in_pad, x, net->Xb);
  gemm(net, (int)n, H, net->in_pad, net->Xb, net->in_pad, 0, net->W1b, H, 0, net->Z1, H);
  hipLaunchKernelGGL(k_bias_relu, dim3(blocks(n * H)), dim3(256), 0, net->stream, n, H, net->Z1,
                     net->P + net->ob1, net->H1b);
  gemm(net, (int)n, H, H, net->H1b, H, 0, net->W2b, H, 0, net->Z2, H);
  hipLaunchKernelGGL(k_bias_relu, dim3(blocks(n * H)), dim3(256), 0, net->stream, n, H, net->Z2,
                     net->P + net->ob2, net->H2b);
  gemm(net, (int)n, net->out_pad, H, net->H2b, H, 0, net->W3b, net->out_pad, 0, net->Zy,
       net->out_pad);
}

// Loss and parameter gradient G for the rows of the last forward pass.
void backward(gq_mlp *net, int64_t n, const float *t, const float *w) {
  const int H = net->n_h, OP = net->out_pad;
  hipLaunchKernelGGL(k_output, dim3(blocks(n * net->n_out)), dim3(256), 0, net->stream, n,
                     net->n_out, OP, net->Zy, net->P + net->ob3, net->Ytmp);
  const float scale = 1.0f / (float)(n * net->n_out);
  hipLaunchKernelGGL(k_loss_grad, dim3(blocks(n * OP)), dim3(256), 0, net->stream, n, net->n_out, OP,
                     net->Ytmp, t, w, scale, net->dY, net->dYb, net->part);
  // layer 3: dW3 = H2^T dY, db3 = colsum dY, dH2 = dY W3^T
  gemm_splitk(net, H, net->n_out, (int)n, net->H2b, H, 1, net->dYb, OP, 0, net->G + net->oW3);
  hipLaunchKernelGGL(k_colsum, dim3(net->n_out), dim3(256), 0, net->stream, n, OP, net->dY,
                     net->G + net->ob3);
  gemm(net, (int)n, H, OP, net->dYb, OP, 0, net->W3b, OP, 1, net->dH, H);
  hipLaunchKernelGGL(k_relu_back, dim3(blocks(n * H)), dim3(256), 0, net->stream, n, H, net->dH,
                     net->Z2, net->dZ, net->dZb);
  // layer 2
  gemm_splitk(net, H, H, (int)n, net->H1b, H, 1, net->dZb, H, 0, net->G + net->oW2);
  hipLaunchKernelGGL(k_colsum, dim3(H), dim3(256), 0, net->stream, n, H, net->dZ, net->G + net->ob2);
  gemm(net, (int)n, H, H, net->dZb, H, 0, net->W2b, H, 1, net->dH, H);
  hipLaunchKernelGGL(k_relu_back, dim3(blocks(n * H)), dim3(256), 0, net->stream, n, H, net->dH,
                     net->Z1, net->dZ, net->dZb);
  // layer 1
  gemm_splitk(net, net->n_in, H, (int)n, net->Xb, net->in_pad, 1, net->dZb, H, 0, net->G + net->oW1);
  hipLaunchKernelGGL(k_colsum, dim3(H), dim3(256), 0, net->stream, n, H, net->dZ, net->G + net->ob1);
}

gq_status read_loss(gq_mlp *net, int64_t n, float *loss) {
  const int64_t nb = (n * net->out_pad + 255) / 256;
  std::vector<float> h(nb);
  GQ_MLP_HIP(net, hipMemcpyAsync(h.data(), net->part, sizeof(float) * nb, hipMemcpyDeviceToHost,
                                 net->stream));
  GQ_MLP_HIP(net, hipStreamSynchronize(net->stream));
  double s = 0.0;
  for (float v : h) s += v;
  *loss = (float)(s / (double)(n * net->n_out));
  return GQ_OK;
}

}  // namespace

extern "C" {

gq_status gq_mlp_create(gq_mlp **out, int device, void *hip_stream, int n_in, int n_hidden,
                        int n_out, uint64_t seed) {
  if (!out) return GQ_EINVAL;
  *out = nullptr;
  if (n_in < 1 || n_in > 64 || n_out < 1 || n_out > 64 || n_hidden < 16 || n_hidden > 256 ||
      n_hidden % 16)
    return GQ_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return GQ_EHIP;
  gq_mlp *net = new (std::nothrow) gq_mlp();
  if (!net) return GQ_ENOMEM;
  net->device = device;
  net->stream = static_cast<hipStream_t>(hip_stream);
  net->n_in = n_in; net->n_h = n_hidden; net->n_out = n_out;
  net->in_pad = pad16(n_in); net->out_pad = pad16(n_out);
  const int64_t H = n_hidden;
  net->oW1 = 0; net->ob1 = n_in * H; net->oW2 = net->ob1 + H; net->ob2 = net->oW2 + H * H;
  net->oW3 = net->ob2 + H; net->ob3 = net->oW3 + H * n_out; net->np = net->ob3 + n_out;
  std::vector<void *> own;
  gq_status s = GQ_OK;
  if (s == GQ_OK) s = dalloc(net, net->P, net->np, own);
  if (s == GQ_OK) s = dalloc(net, net->G, net->np, own);
  if (s == GQ_OK) s = dalloc(net, net->Mo, net->np, own);
  if (s == GQ_OK) s = dalloc(net, net->Vo, net->np, own);
  if (s == GQ_OK) s = dalloc(net, net->W1b, (size_t)net->in_pad * H, own);
  if (s == GQ_OK) s = dalloc(net, net->W2b, (size_t)H * H, own);
  if (s == GQ_OK) s = dalloc(net, net->W3b, (size_t)H * net->out_pad, own);
  if (s != GQ_OK) {
    for (void *p : own) (void)hipFree(p);
    delete net;
    return s;
  }
  // seeded Glorot-uniform initialisation (splitmix64 stream)
  std::vector<float> p(net->np, 0.f);
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int64_t off, int64_t rows, int64_t cols) {
    const double a = std::sqrt(6.0 / (double)(rows + cols));
    for (int64_t i = 0; i < rows * cols; ++i) p[off + i] = (float)((2.0 * next() - 1.0) * a);
  };
  fill(net->oW1, n_in, H);
  fill(net->oW2, H, H);
  fill(net->oW3, H, n_out);
  // the parameter buffers are released by gq_mlp_destroy
  s = gq_mlp_set_params(net, p.data());
  if (s != GQ_OK) {
    gq_mlp_destroy(net);
    return s;
  }
  *out = net;
  return GQ_OK;
}

gq_status gq_mlp_destroy(gq_mlp *net) {
  if (!net) return GQ_OK;
  (void)hipSetDevice(net->device);
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  for (void *p : net->ws) (void)hipFree(p);
  for (void *p : {(void *)net->P, (void *)net->G, (void *)net->Mo, (void *)net->Vo, (void *)net->W1b,
                  (void *)net->W2b, (void *)net->W3b})
    if (p) (void)hipFree(p);
  delete net;
  return GQ_OK;
}

int64_t gq_mlp_param_count(const gq_mlp *net) { return net ? net->np : 0; }

gq_status gq_mlp_shape(const gq_mlp *net, int *n_in, int *n_hidden, int *n_out) {
  if (!net) return GQ_EINVAL;
  if (n_in) *n_in = net->n_in;
  if (n_hidden) *n_hidden = net->n_h;
  if (n_out) *n_out = net->n_out;
  return GQ_OK;
}

gq_status gq_mlp_set_params(gq_mlp *net, const float *host_params) {
  if (!net || !host_params) return mfail(net, GQ_EINVAL, "null argument");
  GQ_MLP_HIP(net, hipSetDevice(net->device));
  GQ_MLP_HIP(net, hipMemcpy(net->P, host_params, sizeof(float) * net->np, hipMemcpyHostToDevice));
  GQ_MLP_HIP(net, hipMemset(net->Mo, 0, sizeof(float) * net->np));
  GQ_MLP_HIP(net, hipMemset(net->Vo, 0, sizeof(float) * net->np));
  net->step = 0;
  refresh_bf16(net);
  GQ_MLP_HIP(net, hipGetLastError());
  GQ_MLP_HIP(net, hipStreamSynchronize(net->stream));
  return GQ_OK;
}

gq_status gq_mlp_get_params(gq_mlp *net, float *host_params) {
  if (!net || !host_params) return mfail(net, GQ_EINVAL, "null argument");
  GQ_MLP_HIP(net, hipSetDevice(net->device));
  GQ_MLP_HIP(net, hipStreamSynchronize(net->stream));
  GQ_MLP_HIP(net, hipMemcpy(host_params, net->P, sizeof(float) * net->np, hipMemcpyDeviceToHost));
  return GQ_OK;
}

gq_status gq_mlp_forward(gq_mlp *net, int64_t n, const float *x, float *y) {
  if (!net) return GQ_EINVAL;
  if (n < 0 || (n > 0 && (!x || !y))) return mfail(net, GQ_EINVAL, "bad rows or null array");
  if (n == 0) return GQ_OK;
  if (n > (int64_t(1) << 26)) return mfail(net, GQ_EUNSUP, "too many rows");
  GQ_MLP_HIP(net, hipSetDevice(net->device));
  gq_status s = ensure_batch(net, n);
  if (s != GQ_OK) return s;
  forward(net, n, x);
  hipLaunchKernelGGL(k_output, dim3(blocks(n * net->n_out)), dim3(256), 0, net->stream, n, net->n_out,
                     net->out_pad, net->Zy, net->P + net->ob3, y);
  GQ_MLP_HIP(net, hipGetLastError());
  return GQ_OK;
}

gq_status gq_mlp_gradients(gq_mlp *net, int64_t n, const float *x, const float *t, const float *w,
                           float *grads, float *loss) {
  if (!net) return GQ_EINVAL;
  if (n <= 0 || !x || !t || !grads) return mfail(net, GQ_EINVAL, "bad rows or null array");
  if (n > (int64_t(1) << 26)) return mfail(net, GQ_EUNSUP, "too many rows");
  GQ_MLP_HIP(net, hipSetDevice(net->device));
  gq_status s = ensure_batch(net, n);
  if (s != GQ_OK) return s;
  forward(net, n, x);
  backward(net, n, t, w);
  GQ_MLP_HIP(net, hipGetLastError());
  if (loss) {
    s = read_loss(net, n, loss);
    if (s != GQ_OK) return s;
  }
  GQ_MLP_HIP(net, hipStreamSynchronize(net->stream));
  GQ_MLP_HIP(net, hipMemcpy(grads, net->G, sizeof(float) * net->np, hipMemcpyDeviceToHost));
  return GQ_OK;
}

gq_status gq_mlp_train_step(gq_mlp *net, int64_t n, const float *x, const float *t, const float *w,
                            float lr, float *loss) {
  if (!net) return GQ_EINVAL;
  if (n <= 0 || !x || !t) return mfail(net, GQ_EINVAL, "bad rows or null array");
  if (n > (int64_t(1) << 26)) return mfail(net, GQ_EUNSUP, "too many rows");
  GQ_MLP_HIP(net, hipSetDevice(net->device));
  gq_status s = ensure_batch(net, n);
  if (s != GQ_OK) return s;
  forward(net, n, x);
  backward(net, n, t, w);
  net->step += 1;
  const float c1 = 1.0f / (1.0f - std::pow(0.9f, (float)net->step));
  const float c2 = 1.0f / (1.0f - std::pow(0.999f, (float)net->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks(net->np)), dim3(256), 0, net->stream, net->np, net->P, net->G,
                     net->Mo, net->Vo, lr, c1, c2);
  refresh_bf16(net);
  GQ_MLP_HIP(net, hipGetLastError());
  if (loss) return read_loss(net, n, loss);
  return GQ_OK;
}

const char *gq_mlp_last_error(gq_mlp *net) { return net ? net->err.c_str() : "null network"; }

void *gq_mlp_stream(const gq_mlp *net) { return net ? static_cast<void *>(net->stream) : nullptr; }

}  // extern "C"
