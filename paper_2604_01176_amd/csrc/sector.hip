// Sector objects (Omega_CIk addressing), error plumbing, FP64-accumulated
// inner products.
#include "hyp_internal.h"

#include <algorithm>
#include <cstring>
#include <new>

namespace hyp {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

hyp_status fail(hyp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

hyp_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HYP_ERR_HIP;
}

static int64_t choose(int m, int k) {
  if (k < 0 || m < 0 || k > m) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (m - k + i) / i;
  return r;
}

// Split colex rank tables for k-subsets of {0..M-1} (see RankTables).
static void make_rank_tables(int M, int k, RankTables* t) {
  for (int v = 0; v < 256; ++v) {
    int n = 0;
    int64_t r = 0;
    for (int b = 0; b < 8; ++b)
      if (v & (1 << b)) r += choose(b, ++n);
    t->lo[v] = (n <= k) ? (int32_t)r : 0;
    int nh = __builtin_popcount(v);
    int kl = k - nh;
    r = 0;
    n = 0;
    if (kl >= 0 && (M > 8 || v == 0)) {
      for (int b = 0; b < 8; ++b)
        if (v & (1 << b)) r += choose(8 + b, kl + (++n));
      t->hi[v] = (int32_t)r;
    } else {
      t->hi[v] = 0;
    }
  }
}

static inline int64_t host_rank(const RankTables& t, uint32_t s) {
  return (int64_t)t.lo[s & 255u] + t.hi[(s >> 8) & 255u];
}

__global__ void k_dot_partial_f64(const double* __restrict__ a, const double* __restrict__ b,
                                  int64_t n, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc = fma(a[i], b[i], acc);
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

__global__ void k_dot_partial_f32(const float* __restrict__ a, const float* __restrict__ b,
                                  int64_t n, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)(a[i] * b[i]);  // FP32 product, FP64 accumulation
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

// Fixed-order final sum of the partials (deterministic, atomic-free).
__global__ void k_sum_partials(const double* __restrict__ part, int n, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    *out = s;
  }
}

hyp_status launch_dot(Sector* S, hyp_dtype dt, const void* a, const void* b, double* out,
                      hipStream_t st) {
  int64_t n = S->dim;
  int blocks = (int)std::min<int64_t>(kDotBlocks, (n + 255) / 256);
  if (blocks < 1) blocks = 1;
  if (dt == HYP_F64)
    HYP_LAUNCH("k_dot_partial_f64", k_dot_partial_f64, dim3(blocks), dim3(256), 0, st, (const double*)a,
                       (const double*)b, n, S->d_scratch);
  else
    HYP_LAUNCH("k_dot_partial_f32", k_dot_partial_f32, dim3(blocks), dim3(256), 0, st, (const float*)a,
                       (const float*)b, n, S->d_scratch);
  HYP_LAUNCH("k_sum_partials", k_sum_partials, dim3(1), dim3(256), 0, st, S->d_scratch, blocks, out);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

}  // namespace hyp

using namespace hyp;

struct hyp_sector_s {
  Sector s;
};

extern "C" {

const char* hyp_last_error(void) { return g_err.c_str(); }

hyp_status hyp_sector_create(int n_orb, int n_alpha, int n_beta, hyp_sector* out) {
  if (!out) return fail(HYP_ERR_ARG, "hyp_sector_create: out is NULL");
  if (n_orb < 1 || n_orb > kMaxOrb)
    return fail(HYP_ERR_SECTOR, "hyp_sector_create: n_orb must be in [1, 16]");
  if (n_alpha < 0 || n_alpha > n_orb || n_beta < 0 || n_beta > n_orb)
    return fail(HYP_ERR_SECTOR, "hyp_sector_create: electron count outside [0, n_orb]");
  hyp_sector_s* h = new (std::nothrow) hyp_sector_s();
  if (!h) return fail(HYP_ERR_NOMEM, "hyp_sector_create: host allocation");
  Sector& S = h->s;
  S.M = n_orb;
  S.na = n_alpha;
  S.nb = n_beta;
  S.da = choose(n_orb, n_alpha);
  S.db = choose(n_orb, n_beta);
  S.dim = S.da * S.db;
  make_rank_tables(n_orb, n_alpha, &S.h_arank);
  make_rank_tables(n_orb, n_beta, &S.h_brank);
  for (uint32_t v = 0; v < (1u << n_orb); ++v) {
    int p = __builtin_popcount(v);
    if (p == n_alpha) S.h_astr.push_back(v);
    if (p == n_beta) S.h_bstr.push_back(v);
  }
  // self-check: ascending enumeration position == split colex rank
  for (size_t i = 0; i < S.h_astr.size(); ++i)
    if (host_rank(S.h_arank, S.h_astr[i]) != (int64_t)i) {
      delete h;
      return fail(HYP_ERR_UNSUPPORTED, "hyp_sector_create: internal rank table check failed");
    }
  hipError_t e;
  (void)hipGetDevice(&S.device);
  e = hipMalloc(&S.d_astr, S.da * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&S.d_bstr, S.db * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&S.d_arank, sizeof(RankTables));
  if (e == hipSuccess) e = hipMalloc(&S.d_brank, sizeof(RankTables));
  if (e == hipSuccess) e = hipMalloc(&S.d_scratch, kScratch * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(S.d_astr, S.h_astr.data(), S.da * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(S.d_bstr, S.h_bstr.data(), S.db * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(S.d_arank, &S.h_arank, sizeof(RankTables), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(S.d_brank, &S.h_brank, sizeof(RankTables), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hyp_sector_destroy(h);
    return hip_fail(e, "hyp_sector_create: device upload");
  }
  *out = h;
  return HYP_OK;
}

hyp_status hyp_sector_destroy(hyp_sector h) {
  if (!h) return HYP_OK;
  Sector& S = h->s;
  (void)hipFree(S.d_astr);
  (void)hipFree(S.d_bstr);
  (void)hipFree(S.d_arank);
  (void)hipFree(S.d_brank);
  (void)hipFree(S.d_scratch);
  (void)hipFree(S.d_pair);
  delete h;
  return HYP_OK;
}

int64_t hyp_sector_dim(hyp_sector h) { return h ? h->s.dim : -1; }

hyp_status hyp_sector_rank(hyp_sector h, const uint32_t* bits, int64_t n, int64_t* idx) {
  if (!h || (n > 0 && (!bits || !idx)) || n < 0)
    return fail(HYP_ERR_ARG, "hyp_sector_rank: NULL argument or negative n");
  const Sector& S = h->s;
  uint32_t am = (1u << S.M) - 1u;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t b = bits[i];
    uint32_t a = b & am, be = b >> S.M;
    if ((S.M < 16 && (be >> S.M)) || __builtin_popcount(a) != S.na ||
        __builtin_popcount(be) != S.nb) {
      idx[i] = -1;
      continue;
    }
    idx[i] = host_rank(S.h_brank, be) * S.da + host_rank(S.h_arank, a);
  }
  return HYP_OK;
}

hyp_status hyp_sector_unrank(hyp_sector h, const int64_t* idx, int64_t n, uint32_t* bits) {
  if (!h || (n > 0 && (!bits || !idx)) || n < 0)
    return fail(HYP_ERR_ARG, "hyp_sector_unrank: NULL argument or negative n");
  const Sector& S = h->s;
  for (int64_t i = 0; i < n; ++i)
    if (idx[i] < 0 || idx[i] >= S.dim) return fail(HYP_ERR_ARG, "hyp_sector_unrank: index out of range");
  for (int64_t i = 0; i < n; ++i)
    bits[i] = S.h_astr[idx[i] % S.da] | (S.h_bstr[idx[i] / S.da] << S.M);
  return HYP_OK;
}

hyp_status hyp_expectation(hyp_sector h, hyp_dtype dtype, const void* a, const void* b,
                           double* out, void* stream) {
  if (!h || !a || !b || !out) return fail(HYP_ERR_ARG, "hyp_expectation: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_expectation: bad dtype");
  return launch_dot(&h->s, dtype, a, b, out, (hipStream_t)stream);
}

}  // extern "C"

namespace hyp {
Sector* sector_of(hyp_sector h) { return h ? &h->s : nullptr; }

// Grow-only scratch for chunk partials.  Growing synchronises the device;
// a call sequence that is captured into a graph must not need to grow it.
hyp_status pair_scratch(Sector* S, size_t n_doubles, double** out) {
  if (n_doubles > S->pair_cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (S->d_pair) HYP_HIP(hipFree(S->d_pair));
    S->d_pair = nullptr;
    S->pair_cap = 0;
    size_t cap = std::max<size_t>(n_doubles, 65536);
    HYP_HIP(hipMalloc(&S->d_pair, cap * sizeof(double)));
    S->pair_cap = cap;
  }
  *out = S->d_pair;
  return HYP_OK;
}
}  // namespace hyp
