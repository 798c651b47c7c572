// order.hip -- learned expansion order per level (2D).
//
// A small multilayer perceptron predicts, for one system and one level k, the
// truncation error that level's far field would carry at each order of a grid
// p = 4..24; the smallest order whose predicted error fits the level's share of
// the tolerance is used.  Features of a (system, level):
//   f0 = k / 10,  f1 = log2(non-empty boxes at level k) / 20,  f2 = log10 ||q||_2.
// Network: 3 -> 64 ReLU -> 64 ReLU -> 21 linear (predicted log10 errors).
// Parameters, one FP32 array (row-major, output index major):
//   W1[64][3], b1[64], W2[64][64], b2[64], W3[21][64], b3[21].
// Training minimises the mean squared error over the 21 outputs with Adam
// (Kingma and Ba 2015, Algorithm 1); every kernel here is deterministic
// (fixed-order reductions, no floating-point atomics).
//
// One wavefront evaluates one sample at a time with lane j owning hidden unit
// j (64 hidden units = 64 lanes); the weights are staged in LDS with rows padded
// to 65 floats so that both row and column walks are free of bank conflicts.
#include "device_common.h"

namespace sffmm {

constexpr int kNI = 3, kNH = 64, kNO = 21;
// Order selection keeps a margin below each level's budget for the network's
// own error of fit: 0.3 in log10 units (a factor of 2), about the RMS error of
// the packaged model's predictions on its training labels (mean squared loss
// 0.10 in log10^2 units).
constexpr float kOrderMargin = 0.3f;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNI, kOffW2 = kOffB1 + kNH,
              kOffB2 = kOffW2 + kNH * kNH, kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNO * kNH,
              kNParam = kOffB3 + kNO;
static_assert(kNParam == FMM_MLP_NPARAM, "parameter count");
constexpr int kRow = 65;  // padded LDS row

struct MlpLds {
  float w1[kNH * kNI], b1[kNH], w2[kNH * kRow], b2[kNH], w3[kNO * kRow], b3[kNO];
};

__device__ void stage_weights(const float* __restrict__ w, MlpLds& s) {
  for (int e = threadIdx.x; e < kNParam; e += blockDim.x) {
    const float v = w[e];
    if (e < kOffB1) {
      s.w1[e] = v;
    } else if (e < kOffW2) {
      s.b1[e - kOffB1] = v;
    } else if (e < kOffB2) {
      const int r = (e - kOffW2) / kNH, c = (e - kOffW2) % kNH;
      s.w2[r * kRow + c] = v;
    } else if (e < kOffW3) {
      s.b2[e - kOffB2] = v;
    } else if (e < kOffB3) {
      const int r = (e - kOffW3) / kNH, c = (e - kOffW3) % kNH;
      s.w3[r * kRow + c] = v;
    } else {
      s.b3[e - kOffB3] = v;
    }
  }
}

// Orders the LDS writes of a wave before its later LDS reads of other lanes'
// values (all lanes of the wave pass it together).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Forward pass of one sample by one wave (lane = hidden unit).  h1s / h2s are
// the wave's LDS vectors.  Returns output `lane` (valid for lanes < 21).
__device__ __forceinline__ float wave_forward(const MlpLds& s, float x0, float x1, float x2,
                                              float* h1s, float* h2s, float& z1, float& h1,
                                              float& z2, float& h2) {
  const int j = threadIdx.x & 63;
  z1 = s.b1[j] + s.w1[j * 3] * x0 + s.w1[j * 3 + 1] * x1 + s.w1[j * 3 + 2] * x2;
  h1 = z1 > 0.f ? z1 : 0.f;
  h1s[j] = h1;
  wave_sync();
  float a = s.b2[j];
#pragma unroll 16
  for (int i = 0; i < kNH; ++i) a += s.w2[j * kRow + i] * h1s[i];
  z2 = a;
  h2 = z2 > 0.f ? z2 : 0.f;
  h2s[j] = h2;
  wave_sync();
  float y = 0.f;
  if (j < kNO) {
    y = s.b3[j];
#pragma unroll 16
    for (int i = 0; i < kNH; ++i) y += s.w3[j * kRow + i] * h2s[i];
  }
  return y;
}

// ---------------------------------------------------------------------------
// Forward over a batch: y[m][21].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w,
                                                     const float* __restrict__ x, int64_t m,
                                                     float* __restrict__ y) {
  __shared__ MlpLds s;
  __shared__ float hs[4][2][kNH];
  stage_weights(w, s);
  __syncthreads();
  const int wv = threadIdx.x >> 6, j = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t smp = (int64_t)blockIdx.x * 4 + wv; smp < m; smp += nw) {
    float z1, h1, z2, h2;
    const float out = wave_forward(s, x[3 * smp], x[3 * smp + 1], x[3 * smp + 2], hs[wv][0],
                                   hs[wv][1], z1, h1, z2, h2);
    if (j < kNO) y[kNO * smp + j] = out;
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Loss gradient: each wave accumulates the gradient of its samples in
// registers (lane i: column i of W2 and W3, row i of W1, biases), then writes
// one partial vector; a second kernel sums the partials in wave order in FP64.
// ---------------------------------------------------------------------------
constexpr int kGradWaves = 4;          // waves per block
constexpr int kSamplesPerWave = 16;

__global__ __launch_bounds__(256) void k_mlp_grad_partial(const float* __restrict__ w,
                                                          const float* __restrict__ x,
                                                          const float* __restrict__ t, int64_t m,
                                                          float scale, float* __restrict__ part,
                                                          double* __restrict__ part_loss) {
  __shared__ MlpLds s;
  __shared__ float hs[4][4][kNH];  // h1, h2, dy, dz2 per wave
  stage_weights(w, s);
  __syncthreads();
  const int wv = threadIdx.x >> 6, j = threadIdx.x & 63;
  const int64_t gw = (int64_t)blockIdx.x * kGradWaves + wv;
  float* h1s = hs[wv][0];
  float* h2s = hs[wv][1];
  float* dys = hs[wv][2];
  float* dz2s = hs[wv][3];
  float g3[kNO], g2[kNH], g1[kNI];
#pragma unroll
  for (int o = 0; o < kNO; ++o) g3[o] = 0.f;
#pragma unroll
  for (int r = 0; r < kNH; ++r) g2[r] = 0.f;
#pragma unroll
  for (int i = 0; i < kNI; ++i) g1[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
  double loss = 0.0;
  const int64_t s0 = gw * kSamplesPerWave;
  for (int u = 0; u < kSamplesPerWave; ++u) {
    const int64_t smp = s0 + u;
    if (smp >= m) break;
    const float x0 = x[3 * smp], x1 = x[3 * smp + 1], x2 = x[3 * smp + 2];
    float z1, h1, z2, h2;
    const float y = wave_forward(s, x0, x1, x2, h1s, h2s, z1, h1, z2, h2);
    float dy = 0.f;
    if (j < kNO) {
      const float e = y - t[kNO * smp + j];
      loss += (double)e * (double)e;
      dy = 2.f * e * scale;
      gb3 += dy;
    }
    dys[j] = dy;
    wave_sync();
    // output layer: dW3[o][i] += dy_o h2_i (lane i), dh2_i = sum_o W3[o][i] dy_o
    float dh2 = 0.f;
#pragma unroll
    for (int o = 0; o < kNO; ++o) {
      const float d = dys[o];
      g3[o] += d * h2;
      dh2 += s.w3[o * kRow + j] * d;
    }
    const float dz2 = z2 > 0.f ? dh2 : 0.f;
    gb2 += dz2;
    dz2s[j] = dz2;
    wave_sync();
    // second layer: dW2[r][i] += dz2_r h1_i (lane i), dh1_i = sum_r W2[r][i] dz2_r
    float dh1 = 0.f;
#pragma unroll
    for (int r = 0; r < kNH; ++r) {
      const float d = dz2s[r];
      g2[r] += d * h1;
      dh1 += s.w2[r * kRow + j] * d;
    }
    const float dz1 = z1 > 0.f ? dh1 : 0.f;
    gb1 += dz1;
    g1[0] += dz1 * x0;
    g1[1] += dz1 * x1;
    g1[2] += dz1 * x2;
    wave_sync();
  }
  float* pp = part + gw * kNParam;
#pragma unroll
  for (int i = 0; i < kNI; ++i) pp[kOffW1 + j * kNI + i] = g1[i];
  pp[kOffB1 + j] = gb1;
#pragma unroll
  for (int r = 0; r < kNH; ++r) pp[kOffW2 + r * kNH + j] = g2[r];
  pp[kOffB2 + j] = gb2;
#pragma unroll
  for (int o = 0; o < kNO; ++o) pp[kOffW3 + o * kNH + j] = g3[o];
  if (j < kNO) pp[kOffB3 + j] = gb3;
  // wave loss: lanes 0..20 hold the squared errors of their outputs
  for (int d = 32; d >= 1; d >>= 1) loss += __shfl_xor(loss, d, 64);
  if (j == 0) part_loss[gw] = loss;
}

__global__ void k_mlp_grad_reduce(const float* __restrict__ part, const double* __restrict__ part_loss,
                                  int64_t nw, float scale, float* __restrict__ grad,
                                  float* __restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kNParam) {
    double a = 0.0;
    for (int64_t r = 0; r < nw; ++r) a += (double)part[r * kNParam + e];
    grad[e] = (float)a;
  }
  if (e == 0 && loss) {
    double l = 0.0;
    for (int64_t r = 0; r < nw; ++r) l += part_loss[r];
    *loss = (float)(l * (double)scale);
  }
}

// omb1 / omb2 are 1 - beta1 / 1 - beta2 formed in FP64 and rounded once (in FP32
// 1 - 0.999f is 1.3e-5 away from 0.001).
__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ g,
                           float* __restrict__ m1, float* __restrict__ m2, float lr, float beta1,
                           float beta2, float omb1, float omb2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNParam) return;
  const float gi = g[e];
  const float a = beta1 * m1[e] + omb1 * gi;
  const float b = beta2 * m2[e] + omb2 * gi * gi;
  m1[e] = a;
  m2[e] = b;
  w[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

int64_t mlp_grad_waves(int64_t m) { return (m + kSamplesPerWave - 1) / kSamplesPerWave; }

void launch_mlp_forward(const float* w, const float* x, int64_t m, float* y, hipStream_t st) {
  if (m <= 0) return;
  const int64_t blocks = std::min<int64_t>((m + 3) / 4, 4096);
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, st, w, x, m, y);
}

void launch_mlp_grad(const float* w, const float* x, const float* t, int64_t m, float* part,
                     double* part_loss, float* grad, float* loss, hipStream_t st) {
  const float scale = 1.f / (float)(kNO * (m > 0 ? m : 1));
  const int64_t nw = mlp_grad_waves(m);
  if (nw > 0) {
    const int64_t blocks = (nw + kGradWaves - 1) / kGradWaves;
    hipLaunchKernelGGL(k_mlp_grad_partial, dim3((unsigned)blocks), dim3(256), 0, st, w, x, t, m,
                       scale, part, part_loss);
  }
  // waves of the last block beyond nw wrote partials too: include only nw
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, st, part,
                     part_loss, nw, 1.f / (float)(kNO * (m > 0 ? m : 1)), grad, loss);
}

void launch_mlp_adam(float* w, const float* g, float* m1, float* m2, int step, float lr,
                     hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, (double)step));
  const float c2 = (float)(1.0 - std::pow(b2, (double)step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, w, g, m1, m2, lr,
                     (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

// ---------------------------------------------------------------------------
// Order selection inside an evaluation.
//   k_order_partials: block b of system s covers sorted positions
//     [start_s + c * kChunk, ...) with c = b - blk0_s; it counts, for every
//     level, the positions whose level-k box differs from the previous
//     position's (the first position of a system counts too) and sums q^2 in
//     FP64 (fixed order).
//   k_order_select: one block per system sums its chunks in order, forms the
//     features of every level 2..L_s, runs the network (one wave per level) and
//     raises the order of the system's depth group at that level to its choice.
// ---------------------------------------------------------------------------
constexpr int kChunk = 4096;

__global__ __launch_bounds__(256) void k_order_partials(const OrderSys* __restrict__ sys, int nsys,
                                                        const uint32_t* __restrict__ keys,
                                                        const int32_t* __restrict__ perm,
                                                        const double* __restrict__ q, int kbits,
                                                        double* __restrict__ pq,
                                                        int32_t* __restrict__ pcnt,
                                                        const BatchIo* __restrict__ io) {
  if (io) q = io->q;
  // system of this block: last s with blk0 <= blockIdx.x
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].blk0 <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const OrderSys sy = sys[lo];
  const int c = (int)blockIdx.x - sy.blk0;
  const int64_t a = (int64_t)sy.start + (int64_t)c * kChunk;
  const int64_t end = (int64_t)sy.start + sy.n;
  const int64_t e = a + kChunk < end ? a + kChunk : end;
  int cnt[kMaxLevels2D + 1];
#pragma unroll
  for (int k = 0; k <= kMaxLevels2D; ++k) cnt[k] = 0;
  double s2 = 0.0;
  for (int64_t j = a + threadIdx.x; j < e; j += 256) {
    const double qq = q[perm[j]];
    s2 += qq * qq;
    const uint32_t kj = keys[j];
    const bool first = j == sy.start;
    const uint32_t kp = first ? 0u : keys[j - 1];
#pragma unroll
    for (int k = 0; k <= kMaxLevels2D; ++k) {
      if (k <= sy.L) {
        const int sh = 2 * (kbits - k);
        cnt[k] += (first || (kj >> sh) != (kp >> sh)) ? 1 : 0;
      }
    }
  }
  __shared__ double rs[256];
  __shared__ int rc[256];
  rs[threadIdx.x] = s2;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) rs[threadIdx.x] += rs[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) pq[blockIdx.x] = rs[0];
  for (int k = 0; k <= kMaxLevels2D; ++k) {
    __syncthreads();
    rc[threadIdx.x] = cnt[k];
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
      if ((int)threadIdx.x < d) rc[threadIdx.x] += rc[threadIdx.x + d];
      __syncthreads();
    }
    if (threadIdx.x == 0) pcnt[(int64_t)blockIdx.x * (kMaxLevels2D + 1) + k] = rc[0];
  }
}

__global__ __launch_bounds__(256) void k_order_select(const OrderSys* __restrict__ sys,
                                                      const float* __restrict__ w,
                                                      const double* __restrict__ pq,
                                                      const int32_t* __restrict__ pcnt,
                                                      float log10_budget, int32_t* __restrict__ ord,
                                                      int ord_cols, float* __restrict__ feat_out) {
  __shared__ MlpLds s;
  __shared__ float hs[4][2][kNH];
  __shared__ double qsum;
  __shared__ int boxes[kMaxLevels2D + 1];
  stage_weights(w, s);
  const OrderSys sy = sys[blockIdx.x];
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int c = 0; c < sy.nblk; ++c) a += pq[sy.blk0 + c];
    qsum = a;
  }
  if ((int)threadIdx.x <= kMaxLevels2D) {
    int b = 0;
    for (int c = 0; c < sy.nblk; ++c) b += pcnt[(int64_t)(sy.blk0 + c) * (kMaxLevels2D + 1) + threadIdx.x];
    boxes[threadIdx.x] = b;
  }
  __syncthreads();
  if (sy.L < 2 || sy.n == 0) return;
  const int wv = threadIdx.x >> 6, j = threadIdx.x & 63;
  const float qn = (float)log10(fmax(sqrt(qsum), 1e-30));
  // the error budget of one level: tol / (number of levels with a far field),
  // less kOrderMargin for the network's own error of fit
  const float thr = log10_budget - log10f((float)(sy.L - 1)) - kOrderMargin;
  for (int k = 2 + wv; k <= sy.L; k += 4) {
    const float f0 = (float)k / 10.f;
    const float f1 = log2f((float)max(boxes[k], 1)) / 20.f;
    float z1, h1, z2, h2;
    const float y = wave_forward(s, f0, f1, qn, hs[wv][0], hs[wv][1], z1, h1, z2, h2);
    const bool ok = j < kNO && y <= thr;
    const uint64_t mask = __ballot(ok);
    if (j == 0) {
      const int p = mask ? 4 + __builtin_ctzll(mask) : 4 + kNO - 1;
      atomicMax(&ord[sy.group * ord_cols + k], p);
      if (feat_out) {
        float* fo = feat_out + ((int64_t)sy.id * (kMaxLevels2D + 1) + k) * 3;
        fo[0] = f0;
        fo[1] = f1;
        fo[2] = qn;
      }
    }
    wave_sync();
  }
}

void launch_order_select(const OrderSys* sys, int nsys, int total_blocks, const uint32_t* keys,
                         const int32_t* perm, const double* q, int kbits, const float* w,
                         double* pq, int32_t* pcnt, float log10_budget, int32_t* ord, int ord_cols,
                         float* feat_out, hipStream_t st, const BatchIo* io) {
  if (nsys <= 0) return;
  if (total_blocks > 0)
    hipLaunchKernelGGL(k_order_partials, dim3(total_blocks), dim3(256), 0, st, sys, nsys, keys,
                       perm, q, kbits, pq, pcnt, io);
  hipLaunchKernelGGL(k_order_select, dim3(nsys), dim3(256), 0, st, sys, w, pq, pcnt, log10_budget,
                     ord, ord_cols, feat_out);
}

int order_chunk() { return kChunk; }

__global__ void k_set_ordsys(OrderSys* dst, OrderSys v) { *dst = v; }

void launch_set_ordsys(OrderSys* dst, const OrderSys& v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_ordsys, dim3(1), dim3(1), 0, st, dst, v);
}

// ---------------------------------------------------------------------------
// Judge: the relative L2 difference of the potentials from the fixed-order
// result over every particle of each system (one workgroup per system, its
// range of the concatenated arrays), and the largest over the systems; if that
// is above tol, flag[1] = tag and the outputs are replaced by the fixed-order
// result.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_judge_sys(const double* __restrict__ pot,
                                                   const double* __restrict__ ref,
                                                   const int64_t* __restrict__ sys_off, int64_t n,
                                                   double* __restrict__ err_sys) {
  __shared__ double a[256], b[256];
  const int64_t i0 = sys_off ? sys_off[blockIdx.x] : 0;
  const int64_t i1 = sys_off ? sys_off[blockIdx.x + 1] : n;
  double num = 0.0, den = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double d = pot[i] - ref[i];
    num += d * d;
    den += ref[i] * ref[i];
  }
  a[threadIdx.x] = num;
  b[threadIdx.x] = den;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) {
      a[threadIdx.x] += a[threadIdx.x + d];
      b[threadIdx.x] += b[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    err_sys[blockIdx.x] = b[0] > 0 ? sqrt(a[0] / b[0]) : (a[0] > 0 ? INFINITY : 0.0);
}

__global__ __launch_bounds__(256) void k_judge_max(const double* __restrict__ err_sys, int nsys,
                                                   double tol, int32_t* flag, int32_t tag,
                                                   double* __restrict__ err_out) {
  __shared__ double m[256];
  __shared__ int reject;
  if (threadIdx.x == 0) reject = 0;
  __syncthreads();
  double e = 0.0;
  bool bad = false;
  for (int s = threadIdx.x; s < nsys; s += 256) {
    const double v = err_sys[s];
    bad = bad || !(v <= tol);  // NaN rejects too
    e = fmax(e, v);
  }
  if (bad) atomicOr(&reject, 1);
  m[threadIdx.x] = e;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if ((int)threadIdx.x < d) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    err_out[0] = m[0];
    if (reject) flag[1] = tag;
  }
}

__global__ void k_judge_apply(double* __restrict__ pot, double* __restrict__ field,
                              const double* __restrict__ rpot, const double* __restrict__ rfield,
                              int64_t n, int dim, const int32_t* flag, int32_t tag) {
  if (flag[1] != tag) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pot[i] = rpot[i];
  if (field)
    for (int d = 0; d < dim; ++d) field[dim * i + d] = rfield[dim * i + d];
}

void launch_judge(double* pot, double* field, const double* rpot, const double* rfield, int64_t n,
                  int dim, const int64_t* sys_off, int nsys, double tol, int32_t* flag,
                  int32_t tag, double* err_out, hipStream_t st) {
  if (n <= 0 || nsys <= 0) return;
  hipLaunchKernelGGL(k_judge_sys, dim3((unsigned)nsys), dim3(256), 0, st, pot, rpot, sys_off, n,
                     err_out + 1);
  hipLaunchKernelGGL(k_judge_max, dim3(1), dim3(256), 0, st, err_out + 1, nsys, tol, flag, tag,
                     err_out);
  hipLaunchKernelGGL(k_judge_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pot,
                     field, rpot, rfield, n, dim, flag, tag);
}

}  // namespace sffmm
