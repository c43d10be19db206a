// Learned gradient screen: per-operator features, a 3-layer MLP
// (32 -> 256 -> 256 -> 1, BF16 weights and MFMA-fed activations, FP32
// accumulation, FP32 master weights), its backward pass and Adam, and the
// top-K ranking.  The screen only decides which pool gradients are computed
// exactly; the exact gradients (and the full-sweep fallback) come from the
// pool-gradient kernels.
#include "hyp_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace hyp {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __host__ inline uint16_t f2bf(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __host__ inline float bf2f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// ---------------------------------------------------------------- occupations

// part[row][q] = sum over the row's alpha columns of psi^2 [q in alpha] (q < M),
// part[row][M] = row total; one workgroup per beta row.
template <typename T>
__global__ void k_occ_rows(const T* psi, int M, int da, const uint32_t* astr, double* part) {
  const int row = blockIdx.x;
  double acc[kMaxOrb + 1];
#pragma unroll
  for (int q = 0; q <= kMaxOrb; ++q) acc[q] = 0.0;
  for (int c = threadIdx.x; c < da; c += blockDim.x) {
    const double v = (double)psi[(int64_t)row * da + c];
    const double w = v * v;
    const uint32_t s = astr[c];
#pragma unroll
    for (int q = 0; q < kMaxOrb; ++q)
      if (s & (1u << q)) acc[q] += w;
    acc[kMaxOrb] += w;
  }
  __shared__ double red[kMaxOrb + 1][4];
#pragma unroll
  for (int q = 0; q <= kMaxOrb; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x <= kMaxOrb) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[threadIdx.x][w];
    const int q = threadIdx.x;
    if (q < M) part[(int64_t)row * (kMaxOrb + 1) + q] = s;
    if (q == kMaxOrb) part[(int64_t)row * (kMaxOrb + 1) + kMaxOrb] = s;
  }
}

// occ[q] for the 2M spin-orbitals: alpha from column sums, beta from the
// row totals of the rows whose beta string holds q.
__global__ void k_occ_final(const double* part, int M, int db, const uint32_t* bstr, double* occ) {
  const int q = threadIdx.x;
  if (q >= 2 * M) return;
  double s = 0.0;
  if (q < M) {
    for (int r = 0; r < db; ++r) s += part[(int64_t)r * (kMaxOrb + 1) + q];
  } else {
    for (int r = 0; r < db; ++r)
      if (bstr[r] & (1u << (q - M))) s += part[(int64_t)r * (kMaxOrb + 1) + kMaxOrb];
  }
  occ[q] = s;
}

// ---------------------------------------------------------------- features

// X[k][0..31] (BF16) = static features with the dynamic slots filled in:
//   11..14  <n_q> of the operator's spin-orbitals (qidx, -1 -> 0)
//   15      log10(|g_prev| + 1e-12)
//   16      min(age, 50) / 10
struct LastSel {
  int q[4];      // qubit indices of the last selected operator (-1 padding; all -1: none)
  float logg;    // log10(|g| + 1e-12) it was selected with
  int M;         // orbitals
};

__global__ void k_features(const float* stat, const int* qidx, const double* occ,
                           const double* gprev, const int* age, int64_t n, LastSel last, uint16_t* X) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float f[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) f[i] = stat[k * 32 + i];
  uint32_t mk = 0, sk = 0, ml = 0, sl = 0;  // spin-orbital and spatial masks
  bool same = true, any = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = qidx[k * 4 + i];
    f[11 + i] = q >= 0 ? (float)occ[q] : 0.0f;
    if (q >= 0) {
      mk |= 1u << q;
      sk |= 1u << (q % last.M);
    }
    const int ql = last.q[i];
    if (ql >= 0) {
      ml |= 1u << ql;
      sl |= 1u << (ql % last.M);
      any = true;
    }
    same = same && q == ql;
  }
  f[15] = (float)log10(fabs(gprev[k]) + 1e-12);
  f[16] = (float)min(age[k], 50) / 10.0f;
  // the operator against the last selected one: the same operator, the
  // spin-orbitals and the spatial orbitals the two share, the size of the
  // last selection's gradient (0 before the first selection)
  f[18] = (any && same) ? 1.0f : 0.0f;
  f[19] = (float)__popc(mk & ml) / 4.0f;
  f[20] = (float)__popc(sk & sl) / 4.0f;
  f[21] = any ? last.logg : 0.0f;
#pragma unroll
  for (int i = 0; i < 32; ++i) X[k * 32 + i] = f2bf(f[i]);
}

// ---------------------------------------------------------------- MFMA GEMM

struct GemmArgs {
  const uint16_t* A;  // element (m, k) at A[m*sam + k*sak]
  const uint16_t* B;  // element (k, n) at B[k*sbk + n*sbn]
  int64_t sam, sak, sbk, sbn;
  int M, N, K;        // multiples of 16
  const float* bias;  // [N] or null
  int relu;           // apply relu to the stored bf16 copy
  float* C;           // [M][N] fp32 (pre-activation) or null
  uint16_t* Cb;       // [M][N] bf16 (post-activation) or null
};

// 64x64 output tile per 256-thread workgroup; each wave a 32x32 sub-tile of
// four 16x16x32 BF16 MFMAs (gfx950) per 32-wide k-chunk.  The chunk's A tile
// (64 rows x 32 k) and B tile (32 k x 64 columns, stored column-major) are
// staged in LDS with k contiguous, so a lane's 8 operand values are one
// 16-byte LDS read: lane l of an MFMA supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] for j < 8 (the same k slots on both sides, which
// is all the reduction needs) and holds D[4 (l / 16) + i][l % 16].  Rows of
// the LDS tiles are padded to 40 elements (80 bytes) against bank conflicts;
// k past K and rows or columns past M, N are staged as zeros.
constexpr int kGemmLd = 40;
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[64 * kGemmLd];
  __shared__ __align__(16) uint16_t Bs[64 * kGemmLd];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int mw = (wave >> 1) * 32, nw = (wave & 1) * 32;
  const int li = lane & 15, lg = lane >> 4;
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    // stage: 64 x 32 elements of each operand, 8 per thread
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = t * 256 + tid;
      const int r = e >> 5, k = e & 31;
      const int kk = k0 + k;
      const int m = m0 + r, n = n0 + r;
      As[r * kGemmLd + k] = (m < g.M && kk < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)kk * g.sak] : (uint16_t)0;
      Bs[r * kGemmLd + k] = (n < g.N && kk < g.K) ? g.B[(int64_t)kk * g.sbk + (int64_t)n * g.sbn] : (uint16_t)0;
    }
    __syncthreads();
    bf16x8_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *(const bf16x8_t*)&As[(mw + i * 16 + li) * kGemmLd + lg * 8];
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *(const bf16x8_t*)&Bs[(nw + j * 16 + li) * kGemmLd + lg * 8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + nw + j * 16 + li;
      if (n >= g.N) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + mw + i * 16 + lg * 4 + t;
        if (m >= g.M) continue;
        float v = acc[i][j][t] + (g.bias ? g.bias[n] : 0.f);
        if (g.C) g.C[(int64_t)m * g.N + n] = v;
        if (g.Cb) g.Cb[(int64_t)m * g.N + n] = f2bf(g.relu ? fmaxf(v, 0.f) : v);
      }
    }
}

// y[r] = sum_n relu(Z2[r][n]) W3[n] + b3
__global__ void k_mlp_out(const float* Z2, const float* W3, const float* b3, int64_t n, float* y) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  float s = 0.f;
  for (int j = lane; j < 256; j += 64) s += fmaxf(Z2[r * 256 + j], 0.f) * W3[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[r] = s + b3[0];
}

// ---------------------------------------------------------------- backward

// dy = 2 (y - t) / B ; dZ2 = dy W3 [Z2 > 0] (fp32 and bf16)
__global__ void k_mlp_dz2(const float* y, const float* t, const float* Z2, const float* W3, int B,
                          float* dy, float* dZ2, uint16_t* dZ2b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * 256) return;
  const int r = (int)(i / 256), j = (int)(i % 256);
  const float d = 2.f * (y[r] - t[r]) / (float)B;
  if (j == 0) dy[r] = d;
  const float v = Z2[i] > 0.f ? d * W3[j] : 0.f;
  dZ2[i] = v;
  dZ2b[i] = f2bf(v);
}

// dZ1 = dH1 [Z1 > 0] (fp32 and bf16)
__global__ void k_mlp_dz1(const float* dH1, const float* Z1, int64_t n, float* dZ1, uint16_t* dZ1b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = Z1[i] > 0.f ? dH1[i] : 0.f;
  dZ1[i] = v;
  dZ1b[i] = f2bf(v);
}

// column sums: out[j] = sum_r X[r][j] (bias gradients), and dW3 / db3
__global__ void k_colsum(const float* X, int rows, int cols, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(int64_t)r * cols + j];
  out[j] = s;
}
__global__ void k_dw3(const float* dy, const float* Z2, int B, float* dW3, float* db3) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 256) {
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += dy[r] * fmaxf(Z2[(int64_t)r * 256 + j], 0.f);
    dW3[j] = s;
  }
  if (j == 256) {
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += dy[r];
    db3[0] = s;
  }
}

// Adam on FP32 masters; refresh the BF16 copy (if any)
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t* pb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = w;
  if (pb) pb[i] = f2bf(w);
}

__global__ void k_cast_bf16(const float* a, int64_t n, uint16_t* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

// Stable sort of n scores, descending (ties keep index order): one
// workgroup, least-significant-digit radix sort over 8 passes of 4 bits of
// an order-reversing integer image of the FP32 key (keys negated in order:
// descending scores become ascending images; -0 is taken as +0).  Thread t
// owns the index range [t n / T, (t + 1) n / T): per pass it counts its
// digits, an exclusive scan in (digit, thread) order gives every thread its
// first position per digit, and the thread scatters its range in order, so
// equal digits keep their order and the sort is stable.  Keys and indices
// alternate between (uA, iA) and (uB, iB); after the eighth pass they are
// back in (uA, iA), iA being the output order.
constexpr int kSortThreads = 1024;
__global__ void __launch_bounds__(kSortThreads) k_rank_sort(const float* __restrict__ y, const float* __restrict__ base,
                                                           int64_t n, uint32_t* uA, int* iA, uint32_t* uB, int* iB) {
  __shared__ int cnt[16 * kSortThreads];  // [digit][thread], then first positions
  __shared__ int wsum[kSortThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t lo = (int64_t)t * n / kSortThreads, hi = (int64_t)(t + 1) * n / kSortThreads;
  for (int64_t i = lo; i < hi; ++i) {
    float f = y[i] + (base ? base[i] : 0.f);
    uint32_t b = __float_as_uint(f);
    if (b == 0x80000000u) b = 0u;                     // -0 as +0
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);   // ascending image of the float order
    uA[i] = ~b;                                       // descending scores first
    iA[i] = (int)i;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const uint32_t* us = (pass & 1) ? uB : uA;
    const int* is = (pass & 1) ? iB : iA;
    uint32_t* ud = (pass & 1) ? uA : uB;
    int* id = (pass & 1) ? iA : iB;
    const int sh = 4 * pass;
    int c[16];
#pragma unroll
    for (int d = 0; d < 16; ++d) c[d] = 0;
    for (int64_t i = lo; i < hi; ++i) {
      const int d = (us[i] >> sh) & 15;
#pragma unroll
      for (int e = 0; e < 16; ++e) c[e] += (d == e) ? 1 : 0;
    }
#pragma unroll
    for (int d = 0; d < 16; ++d) cnt[d * kSortThreads + t] = c[d];
    __syncthreads();
    // exclusive scan of cnt in flattened (digit, thread) order: thread t owns
    // entries [16 t, 16 t + 16)
    int v[16], s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      v[j] = cnt[16 * t + j];
      s += v[j];
    }
    int inc = s;  // inclusive scan of the per-thread sums across the workgroup
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(inc, o, 64);
      if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int before = 0;
    for (int j = 0; j < w; ++j) before += wsum[j];
    int run = before + inc - s;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      cnt[16 * t + j] = run;
      run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 16; ++d) c[d] = cnt[d * kSortThreads + t];
    for (int64_t i = lo; i < hi; ++i) {
      const uint32_t u = us[i];
      const int d = (u >> sh) & 15;
      int pos = 0;
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (d == e) pos = c[e]++;
      ud[pos] = u;
      id[pos] = is[i];
    }
    __syncthreads();  // this pass's scatter complete before the next pass reads it
  }
}

__global__ void k_iota(int* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

// exact gradients just computed (non-NaN entries of g) become the new
// g_prev with age 0; every other operator ages by one iteration
__global__ void k_screen_update(const double* g, int64_t n, double* gprev, int* age) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = g[k];
  if (v == v) {
    gprev[k] = v;
    age[k] = 0;
  } else {
    age[k] = min(age[k] + 1, 1 << 20);
  }
}

// base[k] = max(log10(|g_prev[k]| + 1e-12), floor): the score the network corrects
__global__ void k_screen_base(const double* gprev, int64_t n, float t_floor, float* base) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  base[k] = fmaxf((float)log10(fabs(gprev[k]) + 1e-12), t_floor);
}

// ranking key = network output + base
__global__ void k_add_base(const float* y, const float* base, int64_t n, float* key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) key[k] = y[k] + base[k];
}

// training rows: Xo[i] = X[idx[i]], t[i] = max(log10(|g[idx[i]]| + 1e-12), floor) - base[idx[i]]
__global__ void k_screen_batch(const uint16_t* X, const double* g, const int* idx, int64_t m,
                               float t_floor, const float* base, uint16_t* Xo, float* t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * 32) return;
  const int64_t r = i / 32, c = i % 32;
  const int64_t k = idx[r];
  Xo[i] = X[k * 32 + c];
  if (c == 0) t[r] = fmaxf((float)log10(fabs(g[k]) + 1e-12), t_floor) - (base ? base[k] : 0.f);
}

static unsigned g1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace hyp

using namespace hyp;

// ---------------------------------------------------------------- C ABI

struct hyp_mlp_s {
  // fp32 masters, Adam moments, grads; bf16 copies of W1, W2
  float *W1, *b1, *W2, *b2, *W3, *b3;
  float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
  float *mW1, *mb1, *mW2, *mb2, *mW3, *mb3;
  float *vW1, *vb1, *vW2, *vb2, *vW3, *vb3;
  uint16_t *W1b, *W2b;
  int64_t cap;               // rows of the activation buffers
  float *Z1, *Z2, *dH1, *dZ1, *dZ2, *dy;
  uint16_t *H1b, *dZ1b, *dZ2b;
  int64_t step;
  void* sort_tmp;
  size_t sort_tmp_bytes;
  int64_t sort_cap;
  float *keys_out, *keys_in;
  int *idx_in, *idx_out;
};

static const int64_t kW1 = 256 * 32, kW2 = 256 * 256, kW3 = 256;

extern "C" {

hyp_status hyp_mlp_create(const float* init_host, int64_t max_rows, hyp_mlp* out) {
  if (!init_host || !out || max_rows < 64) return fail(HYP_ERR_ARG, "hyp_mlp_create: bad argument");
  hyp_mlp_s* m = new (std::nothrow) hyp_mlp_s();
  if (!m) return fail(HYP_ERR_NOMEM, "hyp_mlp_create");
  std::memset(m, 0, sizeof(*m));
  const int64_t np = kW1 + 256 + kW2 + 256 + kW3 + 1;
  m->cap = (max_rows + 63) / 64 * 64;
  float* P = nullptr;
  hipError_t e = hipMalloc(&P, sizeof(float) * np * 4);  // params, grads, m, v
  if (e == hipSuccess) e = hipMemcpy(P, init_host, sizeof(float) * np, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(P + np, 0, sizeof(float) * np * 3);
  auto carve = [&](float* base, float** w1, float** b1, float** w2, float** b2, float** w3, float** b3) {
    *w1 = base; *b1 = base + kW1; *w2 = *b1 + 256; *b2 = *w2 + kW2; *w3 = *b2 + 256; *b3 = *w3 + kW3;
  };
  if (e == hipSuccess) {
    carve(P, &m->W1, &m->b1, &m->W2, &m->b2, &m->W3, &m->b3);
    carve(P + np, &m->gW1, &m->gb1, &m->gW2, &m->gb2, &m->gW3, &m->gb3);
    carve(P + 2 * np, &m->mW1, &m->mb1, &m->mW2, &m->mb2, &m->mW3, &m->mb3);
    carve(P + 3 * np, &m->vW1, &m->vb1, &m->vW2, &m->vb2, &m->vW3, &m->vb3);
  }
  if (e == hipSuccess) e = hipMalloc(&m->W1b, 2 * (kW1 + kW2));
  if (e == hipSuccess) {
    m->W2b = m->W1b + kW1;
    e = hipMalloc(&m->Z1, sizeof(float) * m->cap * 256 * 5 + sizeof(float) * m->cap);
  }
  if (e == hipSuccess) {
    m->Z2 = m->Z1 + m->cap * 256;
    m->dH1 = m->Z2 + m->cap * 256;
    m->dZ1 = m->dH1 + m->cap * 256;
    m->dZ2 = m->dZ1 + m->cap * 256;
    m->dy = m->dZ2 + m->cap * 256;
    e = hipMalloc(&m->H1b, 2 * m->cap * 256 * 3);
  }
  if (e == hipSuccess) {
    m->dZ1b = m->H1b + m->cap * 256;
    m->dZ2b = m->dZ1b + m->cap * 256;
  }
  if (e == hipSuccess) {
    HYP_LAUNCH("k_cast_bf16", k_cast_bf16, dim3(g1(kW1)), dim3(256), 0, 0, m->W1, kW1, m->W1b);
    HYP_LAUNCH("k_cast_bf16", k_cast_bf16, dim3(g1(kW2)), dim3(256), 0, 0, m->W2, kW2, m->W2b);
    e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    hyp_mlp_destroy(m);
    return hip_fail(e, "hyp_mlp_create: allocation");
  }
  *out = m;
  return HYP_OK;
}

hyp_status hyp_mlp_destroy(hyp_mlp m) {
  if (!m) return HYP_OK;
  (void)hipFree(m->W1);
  (void)hipFree(m->W1b);
  (void)hipFree(m->Z1);
  (void)hipFree(m->H1b);
  (void)hipFree(m->sort_tmp);
  (void)hipFree(m->keys_out);
  (void)hipFree(m->keys_in);
  (void)hipFree(m->idx_in);
  (void)hipFree(m->idx_out);
  delete m;
  return HYP_OK;
}

hyp_status hyp_mlp_params(hyp_mlp m, float* host_out) {
  if (!m || !host_out) return fail(HYP_ERR_ARG, "hyp_mlp_params: NULL argument");
  const int64_t np = kW1 + 256 + kW2 + 256 + kW3 + 1;
  HYP_HIP(hipDeviceSynchronize());
  HYP_HIP(hipMemcpy(host_out, m->W1, sizeof(float) * np, hipMemcpyDeviceToHost));
  return HYP_OK;
}

static hyp_status mlp_forward(hyp_mlp m, const uint16_t* X, int64_t n, float* y, hipStream_t st) {
  const int64_t np = (n + 63) / 64 * 64;
  GemmArgs g{};
  // Z1 = X W1^T + b1 ; H1 = bf16(relu(Z1))
  g.A = X; g.sam = 32; g.sak = 1;
  g.B = m->W1b; g.sbk = 1; g.sbn = 32;
  g.M = (int)n; g.N = 256; g.K = 32; g.bias = m->b1; g.relu = 1; g.C = m->Z1; g.Cb = m->H1b;
  HYP_LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3(4, (unsigned)(np / 64)), dim3(256), 0, st, g);
  // Z2 = H1 W2^T + b2
  g.A = m->H1b; g.sam = 256; g.sak = 1;
  g.B = m->W2b; g.sbk = 1; g.sbn = 256;
  g.K = 256; g.bias = m->b2; g.relu = 0; g.C = m->Z2; g.Cb = nullptr;
  HYP_LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3(4, (unsigned)(np / 64)), dim3(256), 0, st, g);
  HYP_LAUNCH("k_mlp_out", k_mlp_out, dim3(g1(n, 4)), dim3(256), 0, st, m->Z2, m->W3, m->b3, n, y);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

// scores y[n] (device) for feature rows X (device bf16 [n][32]); n <= max_rows
hyp_status hyp_mlp_forward(hyp_mlp m, const uint16_t* X_dev, int64_t n, float* y_dev, void* stream) {
  if (!m || !X_dev || !y_dev || n < 1 || n > m->cap) return fail(HYP_ERR_ARG, "hyp_mlp_forward: bad argument");
  return mlp_forward(m, X_dev, n, y_dev, (hipStream_t)stream);
}

// One training step on a batch (B rows, B <= max_rows, multiple of 16):
// forward, MSE loss gradient against targets t, backward, Adam.
// Gradients stay readable through hyp_mlp_grads until the next step.
hyp_status hyp_mlp_train_step(hyp_mlp m, const uint16_t* X_dev, const float* t_dev, int64_t B,
                              float lr, float* y_dev, void* stream) {
  if (!m || !X_dev || !t_dev || !y_dev || B < 16 || B > m->cap || (B % 16))
    return fail(HYP_ERR_ARG, "hyp_mlp_train_step: bad argument");
  if (!(lr > 0)) return fail(HYP_ERR_ARG, "hyp_mlp_train_step: lr must be > 0");
  hipStream_t st = (hipStream_t)stream;
  hyp_status r = mlp_forward(m, X_dev, B, y_dev, st);
  if (r != HYP_OK) return r;
  const int64_t nb = (int64_t)B * 256;
  HYP_LAUNCH("k_mlp_dz2", k_mlp_dz2, dim3(g1(nb)), dim3(256), 0, st, y_dev, t_dev, m->Z2, m->W3, (int)B,
             m->dy, m->dZ2, m->dZ2b);
  HYP_LAUNCH("k_dw3", k_dw3, dim3(2), dim3(256), 0, st, m->dy, m->Z2, (int)B, m->gW3, m->gb3);
  HYP_LAUNCH("k_colsum", k_colsum, dim3(1), dim3(256), 0, st, m->dZ2, (int)B, 256, m->gb2);
  GemmArgs g{};
  // dW2 = dZ2^T H1   [256 x 256], K = B
  g.A = m->dZ2b; g.sam = 1; g.sak = 256;
  g.B = m->H1b; g.sbk = 256; g.sbn = 1;
  g.M = 256; g.N = 256; g.K = (int)B; g.C = m->gW2;
  HYP_LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3(4, 4), dim3(256), 0, st, g);
  // dH1 = dZ2 W2     [B x 256], K = 256
  g.A = m->dZ2b; g.sam = 256; g.sak = 1;
  g.B = m->W2b; g.sbk = 256; g.sbn = 1;
  g.M = (int)B; g.N = 256; g.K = 256; g.C = m->dH1;
  HYP_LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3(4, (unsigned)((B + 63) / 64)), dim3(256), 0, st, g);
  HYP_LAUNCH("k_mlp_dz1", k_mlp_dz1, dim3(g1(nb)), dim3(256), 0, st, m->dH1, m->Z1, nb, m->dZ1, m->dZ1b);
  HYP_LAUNCH("k_colsum", k_colsum, dim3(1), dim3(256), 0, st, m->dZ1, (int)B, 256, m->gb1);
  // dW1 = dZ1^T X    [256 x 32], K = B
  g.A = m->dZ1b; g.sam = 1; g.sak = 256;
  g.B = X_dev; g.sbk = 32; g.sbn = 1;
  g.M = 256; g.N = 32; g.K = (int)B; g.C = m->gW1;
  HYP_LAUNCH("k_gemm_bf16", k_gemm_bf16, dim3(1, 4), dim3(256), 0, st, g);
  // Adam (lr, 0.9, 0.999, 1e-8), bias-corrected
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
  struct P {
    float *p, *g, *mm, *vv;
    int64_t n;
    uint16_t* pb;
  } ps[6] = {{m->W1, m->gW1, m->mW1, m->vW1, kW1, m->W1b}, {m->b1, m->gb1, m->mb1, m->vb1, 256, nullptr},
             {m->W2, m->gW2, m->mW2, m->vW2, kW2, m->W2b}, {m->b2, m->gb2, m->mb2, m->vb2, 256, nullptr},
             {m->W3, m->gW3, m->mW3, m->vW3, kW3, nullptr}, {m->b3, m->gb3, m->mb3, m->vb3, 1, nullptr}};
  for (auto& p : ps)
    HYP_LAUNCH("k_adam", k_adam, dim3(g1(p.n)), dim3(256), 0, st, p.p, p.g, p.mm, p.vv, p.n, lr, b1, b2,
               1e-8f, c1, c2, p.pb);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

// Gradients of the last training step, host layout = parameter layout.
// Full training state: parameters, Adam first and second moments (each in
// the parameter layout) and the Adam step count (one float), 3 np + 1 floats.
hyp_status hyp_mlp_get_state(hyp_mlp m, float* host_out) {
  if (!m || !host_out) return fail(HYP_ERR_ARG, "hyp_mlp_get_state: NULL argument");
  const int64_t np = kW1 + 256 + kW2 + 256 + kW3 + 1;
  HYP_HIP(hipDeviceSynchronize());
  HYP_HIP(hipMemcpy(host_out, m->W1, sizeof(float) * np, hipMemcpyDeviceToHost));
  HYP_HIP(hipMemcpy(host_out + np, m->mW1, sizeof(float) * np, hipMemcpyDeviceToHost));
  HYP_HIP(hipMemcpy(host_out + 2 * np, m->vW1, sizeof(float) * np, hipMemcpyDeviceToHost));
  host_out[3 * np] = (float)m->step;
  return HYP_OK;
}

hyp_status hyp_mlp_set_state(hyp_mlp m, const float* host_in) {
  if (!m || !host_in) return fail(HYP_ERR_ARG, "hyp_mlp_set_state: NULL argument");
  const int64_t np = kW1 + 256 + kW2 + 256 + kW3 + 1;
  const float st = host_in[3 * np];
  if (!(st >= 0.f) || st > 1e9f || st != (float)(int64_t)st)
    return fail(HYP_ERR_ARG, "hyp_mlp_set_state: bad step count");
  HYP_HIP(hipDeviceSynchronize());
  HYP_HIP(hipMemcpy(m->W1, host_in, sizeof(float) * np, hipMemcpyHostToDevice));
  HYP_HIP(hipMemcpy(m->mW1, host_in + np, sizeof(float) * np, hipMemcpyHostToDevice));
  HYP_HIP(hipMemcpy(m->vW1, host_in + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice));
  m->step = (int64_t)st;
  HYP_LAUNCH("k_cast_bf16", k_cast_bf16, dim3(g1(kW1)), dim3(256), 0, 0, m->W1, kW1, m->W1b);
  HYP_LAUNCH("k_cast_bf16", k_cast_bf16, dim3(g1(kW2)), dim3(256), 0, 0, m->W2, kW2, m->W2b);
  HYP_HIP(hipDeviceSynchronize());
  return HYP_OK;
}

hyp_status hyp_mlp_grads(hyp_mlp m, float* host_out) {
  if (!m || !host_out) return fail(HYP_ERR_ARG, "hyp_mlp_grads: NULL argument");
  const int64_t np = kW1 + 256 + kW2 + 256 + kW3 + 1;
  HYP_HIP(hipDeviceSynchronize());
  HYP_HIP(hipMemcpy(host_out, m->gW1, sizeof(float) * np, hipMemcpyDeviceToHost));
  return HYP_OK;
}

// Static feature rows of an operator pool (host): class one-hot, orbital
// indices / (M - 1), log10 of the integral magnitudes, M / 16; and each
// operator's spin-orbital indices (c1, c2, a1, a2; -1 padding).
hyp_status hyp_screen_static(int n_orb, const hyp_exc* pool, const uint8_t* cls, int64_t n,
                             const double* h, const double* g, float* stat, int32_t* qidx) {
  if (n_orb < 1 || n_orb > kMaxOrb || !pool || !cls || !h || !g || !stat || !qidx || n < 0)
    return fail(HYP_ERR_ARG, "hyp_screen_static: bad argument");
  const int M = n_orb;
  const double den = M > 1 ? (double)(M - 1) : 1.0;
  auto G = [&](int p, int q, int r, int s_) { return g[((p * M + q) * M + r) * M + s_]; };
  for (int64_t k = 0; k < n; ++k) {
    float* f = stat + k * 32;
    int32_t* qi = qidx + k * 4;
    for (int i = 0; i < 32; ++i) f[i] = 0.f;
    if (cls[k] > 4) return fail(HYP_ERR_ARG, "hyp_screen_static: class > 4");
    f[cls[k]] = 1.f;
    int cq[2] = {-1, -1}, aq[2] = {-1, -1}, nc = 0, na = 0;
    for (int q = 0; q < 2 * M; ++q) {
      if ((pool[k].cre >> q) & 1u) { if (nc < 2) cq[nc] = q; ++nc; }
      if ((pool[k].ann >> q) & 1u) { if (na < 2) aq[na] = q; ++na; }
    }
    if (nc != na || nc < 1 || nc > 2) return fail(HYP_ERR_ARG, "hyp_screen_static: not a single or double");
    int qs[4];
    if (nc == 1) {
      qs[0] = cq[0]; qs[1] = aq[0]; qs[2] = -1; qs[3] = -1;
      f[9] = (float)std::log10(std::fabs(h[(cq[0] % M) * M + (aq[0] % M)]) + 1e-12);
    } else {
      qs[0] = cq[0]; qs[1] = cq[1]; qs[2] = aq[0]; qs[3] = aq[1];
      const int c1 = cq[0] % M, c2 = cq[1] % M, a1 = aq[0] % M, a2 = aq[1] % M;
      f[9] = (float)std::log10(std::fabs(G(c1, a1, c2, a2)) + 1e-12);
      f[10] = (float)std::log10(std::fabs(G(c1, a2, c2, a1)) + 1e-12);
    }
    for (int i = 0; i < 4; ++i) {
      qi[i] = qs[i];
      f[5 + i] = qs[i] >= 0 ? (float)((qs[i] % M) / den) : -1.f;
    }
    f[17] = (float)(M / 16.0);
  }
  return HYP_OK;
}

// occupations <n_q> (2M doubles, device) of a sector state
hyp_status hyp_occupations(hyp_sector sh, hyp_dtype dt, const void* psi, double* occ_dev,
                           double* work_dev, void* stream) {
  Sector* S = sector_of(sh);
  if (!S || !psi || !occ_dev || !work_dev) return fail(HYP_ERR_ARG, "hyp_occupations: NULL argument");
  hipStream_t st = (hipStream_t)stream;
  if (dt == HYP_F64)
    HYP_LAUNCH("k_occ_rows", k_occ_rows<double>, dim3((unsigned)S->db), dim3(256), 0, st, (const double*)psi,
               S->M, (int)S->da, S->d_astr, work_dev);
  else if (dt == HYP_F32)
    HYP_LAUNCH("k_occ_rows", k_occ_rows<float>, dim3((unsigned)S->db), dim3(256), 0, st, (const float*)psi,
               S->M, (int)S->da, S->d_astr, work_dev);
  else
    return fail(HYP_ERR_ARG, "hyp_occupations: bad dtype");
  HYP_LAUNCH("k_occ_final", k_occ_final, dim3(1), dim3(64), 0, st, work_dev, S->M, (int)S->db, S->d_bstr,
             occ_dev);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_features(const float* stat_dev, const int32_t* qidx_dev, const double* occ_dev,
                        const double* gprev_dev, const int32_t* age_dev, int64_t n, int n_orb,
                        const int32_t* last_qidx, double last_g, uint16_t* X_dev, void* stream) {
  if (!stat_dev || !qidx_dev || !occ_dev || !gprev_dev || !age_dev || !X_dev || !last_qidx || n < 0)
    return fail(HYP_ERR_ARG, "hyp_features: NULL argument");
  if (n_orb < 1 || n_orb > kMaxOrb) return fail(HYP_ERR_ARG, "hyp_features: n_orb out of range");
  LastSel last;
  for (int i = 0; i < 4; ++i) {
    if (last_qidx[i] < -1 || last_qidx[i] >= 2 * n_orb) return fail(HYP_ERR_ARG, "hyp_features: bad last_qidx");
    last.q[i] = last_qidx[i];
  }
  last.logg = (float)std::log10(std::fabs(last_g) + 1e-12);
  last.M = n_orb;
  if (n == 0) return HYP_OK;
  HYP_LAUNCH("k_features", k_features, dim3(g1(n)), dim3(256), 0, (hipStream_t)stream, stat_dev, qidx_dev,
             occ_dev, gprev_dev, age_dev, n, last, X_dev);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_screen_update(const double* g_dev, int64_t n, double* gprev_dev, int32_t* age_dev,
                             void* stream) {
  if (!g_dev || !gprev_dev || !age_dev || n < 0) return fail(HYP_ERR_ARG, "hyp_screen_update: NULL argument");
  if (n == 0) return HYP_OK;
  HYP_LAUNCH("k_screen_update", k_screen_update, dim3(g1(n)), dim3(256), 0, (hipStream_t)stream, g_dev, n,
             gprev_dev, age_dev);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_screen_base(const double* gprev_dev, int64_t n, float t_floor, float* base_dev, void* stream) {
  if (!gprev_dev || !base_dev || n < 0) return fail(HYP_ERR_ARG, "hyp_screen_base: NULL argument");
  if (n == 0) return HYP_OK;
  HYP_LAUNCH("k_screen_base", k_screen_base, dim3(g1(n)), dim3(256), 0, (hipStream_t)stream, gprev_dev, n, t_floor,
             base_dev);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_screen_batch(const uint16_t* X_dev, const double* g_dev, const int32_t* idx_dev, int64_t m,
                            float t_floor, const float* base_dev, uint16_t* Xo_dev, float* t_dev, void* stream) {
  if (!X_dev || !g_dev || !idx_dev || !Xo_dev || !t_dev || m < 0) return fail(HYP_ERR_ARG, "hyp_screen_batch: NULL argument");
  if (m == 0) return HYP_OK;
  HYP_LAUNCH("k_screen_batch", k_screen_batch, dim3(g1(m * 32)), dim3(256), 0, (hipStream_t)stream, X_dev, g_dev,
             idx_dev, m, t_floor, base_dev, Xo_dev, t_dev);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

// order_dev[0..n) = operator indices sorted by descending score (ties: lower index first)
hyp_status hyp_rank_scores(hyp_mlp m, const float* y_dev, const float* base_dev, int64_t n, int32_t* order_dev,
                           void* stream) {
  if (!m || !y_dev || !order_dev || n < 1 || n > (1 << 30)) return fail(HYP_ERR_ARG, "hyp_rank_scores: bad argument");
  hipStream_t st = (hipStream_t)stream;
  if (n > m->sort_cap) {
    HYP_HIP(hipDeviceSynchronize());
    (void)hipFree(m->keys_out);
    (void)hipFree(m->idx_in);
    (void)hipFree(m->keys_in);
    m->keys_out = nullptr;
    m->idx_in = nullptr;
    m->keys_in = nullptr;
    m->sort_cap = 0;
    HYP_HIP(hipMalloc(&m->keys_in, sizeof(uint32_t) * n));
    HYP_HIP(hipMalloc(&m->keys_out, sizeof(uint32_t) * n));
    HYP_HIP(hipMalloc(&m->idx_in, sizeof(int) * n));
    m->sort_cap = n;
  }
  HYP_LAUNCH("k_rank_sort", k_rank_sort, dim3(1), dim3(kSortThreads), 0, st, y_dev, base_dev, n,
             (uint32_t*)m->keys_in, (int*)order_dev, (uint32_t*)m->keys_out, m->idx_in);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

}  // extern "C"
