// Batched pool gradients: every (instance, generator, beta-chunk) work item of
// several uneven-sized problems in one persistent launch.  A grid of
// (CUs x blocks_per_cu) workgroups pops items from a device counter until the
// queue is drained (every wave reaches the exit test), writes one partial per
// item (no atomics on the results), and a second pass sums each generator's
// chunks in a fixed order.  The tile shape (threads per workgroup, chunks per
// generator, resident workgroups per CU) is chosen by hyp_tune_pool_gradients,
// which times the candidates on the actual jobs.
#include "hyp_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace hyp {

constexpr int kMaxJobs = 16;
constexpr int kBListMax = 3432;

__constant__ int c_binom_b[17][17];

struct JobDev {
  SectorDev S;
  const hyp_exc* ops;
  const void* psi;
  const void* sig;
  int64_t n_ops;
  int64_t item_off;    // first work item of this job
  int64_t part_off;    // first partial of this job
};

struct BatchArgs {
  int n_jobs;
  int nch;             // chunks per generator
  int64_t total;       // work items
  int* counter;
  double* part;
  JobDev job[kMaxJobs];
};

__device__ inline int bin_b(int m, int k) { return c_binom_b[m][k]; }

struct BPart {
  uint32_t cm, am, free;
  int count, nsel, nfree;
};

__device__ inline BPart bpart(uint32_t cm, uint32_t am, int M, int N) {
  BPart p;
  p.cm = cm;
  p.am = am;
  p.free = ~(cm | am) & ((1u << M) - 1u);
  p.nfree = __popc(p.free);
  p.nsel = N - __popc(am);
  p.count = (p.nsel < 0 || p.nsel > p.nfree) ? 0 : bin_b(p.nfree, p.nsel);
  return p;
}

__device__ inline uint32_t bpart_string(const BPart& p, int i) {
  uint32_t pos = 0;
  int r = i;
  for (int j = p.nsel; j >= 1; --j) {
    int c = j - 1;
    while (c + 1 < p.nfree && bin_b(c + 1, j) <= r) ++c;
    r -= bin_b(c, j);
    pos |= 1u << c;
  }
  uint32_t s = p.am, f = p.free;
  for (int b = 0; f; ++b) {
    uint32_t low = f & (~f + 1u);
    if (pos & (1u << b)) s |= low;
    f ^= low;
  }
  return s;
}

__device__ inline int bpart_sign(uint32_t cm, uint32_t am, uint32_t s) {
  int odd = 0;
  uint32_t a = am;
  while (a) {
    int q = __ffs(a) - 1;
    a &= a - 1;
    odd += __popc(s & ((1u << q) - 1u));
    s ^= 1u << q;
  }
  uint32_t c = cm;
  while (c) {
    int q = 31 - __clz(c);
    c ^= 1u << q;
    odd += __popc(s & ((1u << q) - 1u));
    s ^= 1u << q;
  }
  return odd & 1;
}

__device__ inline int brank(const RankTables* t, uint32_t s) {
  return t->lo[s & 255u] + t->hi[(s >> 8) & 255u];
}

__global__ void k_reset_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

template <typename T>
__global__ void k_pool_grad_persistent(BatchArgs a) {
  __shared__ uint32_t lst[kBListMax];
  __shared__ double red[16];
  __shared__ int64_t s_item;
  const int nt = blockDim.x;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.counter, 1);
    __syncthreads();
    const int64_t w = s_item;
    __syncthreads();
    if (w >= a.total) break;  // uniform across the workgroup
    int j = 0;
    while (j + 1 < a.n_jobs && a.job[j + 1].item_off <= w) ++j;
    const JobDev& J = a.job[j];
    const int64_t local = w - J.item_off;
    const int64_t k = local / a.nch;
    const int chunk = (int)(local % a.nch);
    const SectorDev& S = J.S;
    const hyp_exc op = J.ops[k];
    const uint32_t m = (1u << S.M) - 1u;
    const BPart pa = bpart(op.cre & m, op.ann & m, S.M, S.na);
    const BPart pb = bpart((op.cre >> S.M) & m, (op.ann >> S.M) & m, S.M, S.nb);
    const bool a_id = (pa.cm | pa.am) == 0, b_id = (pb.cm | pb.am) == 0;
    if (!a_id)
      for (int i = threadIdx.x; i < pa.count; i += nt) {
        uint32_t Js = bpart_string(pa, i);
        uint32_t Is = Js ^ pa.am ^ pa.cm;
        lst[i] = (uint32_t)brank(S.arank, Js) | ((uint32_t)brank(S.arank, Is) << 14) |
                 ((uint32_t)(bpart_sign(pa.cm, pa.am, Js) & S.fsign) << 28);
      }
    __syncthreads();
    const int nA = a_id ? S.da : pa.count;
    const int nB = pb.count;
    const int b0 = (int)((int64_t)nB * chunk / a.nch), b1 = (int)((int64_t)nB * (chunk + 1) / a.nch);
    const T* psi = (const T*)J.psi;
    const T* sig = (const T*)J.sig;
    double acc = 0.0;
    for (int jb = b0; jb < b1; ++jb) {
      int rJb, rIb, sb;
      if (b_id) {
        rJb = rIb = jb;
        sb = 0;
      } else {
        uint32_t Jb = bpart_string(pb, jb);
        uint32_t Ib = Jb ^ pb.am ^ pb.cm;
        rJb = brank(S.brank, Jb);
        rIb = brank(S.brank, Ib);
        sb = bpart_sign(pb.cm, pb.am, Jb) & S.fsign;
      }
      const int64_t oJ = (int64_t)rJb * S.da, oI = (int64_t)rIb * S.da;
      double rs = 0.0;
      for (int t = threadIdx.x; t < nA; t += nt) {
        int rJa, rIa, sa;
        if (a_id) {
          rJa = rIa = t;
          sa = 0;
        } else {
          const uint32_t e = lst[t];
          rJa = e & 0x3fff;
          rIa = (e >> 14) & 0x3fff;
          sa = (e >> 28) & 1;
        }
        const int64_t D = oJ + rJa, Dp = oI + rIa;
        double v;
        if (sizeof(T) == 4)
          v = (double)((float)sig[Dp] * (float)psi[D]) - (double)((float)sig[D] * (float)psi[Dp]);
        else
          v = (double)sig[Dp] * (double)psi[D] - (double)sig[D] * (double)psi[Dp];
        rs += sa ? -v : v;
      }
      acc += sb ? -rs : rs;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int wv = 0; wv < nt / 64; ++wv) s += red[wv];
      a.part[J.part_off + k * a.nch + chunk] = s;
    }
    // the next item overwrites lst and red only after this barrier
    __syncthreads();
  }
}

struct SumArgs {
  int n_jobs, nch;
  int64_t n_off[kMaxJobs + 1];   // generator prefix over jobs
  int64_t part_off[kMaxJobs];
  double* grad[kMaxJobs];
  const double* part;
};

__global__ void k_sum_batched(SumArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.n_off[a.n_jobs]) return;
  int j = 0;
  while (j + 1 < a.n_jobs && a.n_off[j + 1] <= g) ++j;
  const int64_t k = g - a.n_off[j];
  const double* p = a.part + a.part_off[j] + k * a.nch;
  double s = 0.0;
  for (int c = 0; c < a.nch; ++c) s += p[c];
  a.grad[j][k] = 2.0 * s;
}

namespace {
std::mutex g_bmu;
struct BatchScratch {
  double* part = nullptr;
  size_t cap = 0;
  int* counter = nullptr;
  bool binom = false;
};
BatchScratch g_bs[64];
int g_cus[64];
}  // namespace

static hyp_status batch_scratch(size_t n, BatchScratch** out) {
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lk(g_bmu);
  BatchScratch& b = g_bs[dev];
  if (!b.counter) HYP_HIP(hipMalloc(&b.counter, 256));
  if (!b.binom) {
    int tab[17][17];
    for (int mm = 0; mm <= 16; ++mm)
      for (int kk = 0; kk <= 16; ++kk) {
        int64_t r = 0;
        if (kk <= mm) {
          r = 1;
          for (int i = 1; i <= kk; ++i) r = r * (mm - kk + i) / i;
        }
        tab[mm][kk] = (int)r;
      }
    HYP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom_b), tab, sizeof(tab)));
    hipDeviceProp_t prop;
    HYP_HIP(hipGetDeviceProperties(&prop, dev));
    g_cus[dev] = prop.multiProcessorCount;
    b.binom = true;
  }
  if (n > b.cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (b.part) HYP_HIP(hipFree(b.part));
    b.part = nullptr;
    b.cap = 0;
    size_t cap = std::max<size_t>(n, 1 << 16);
    HYP_HIP(hipMalloc(&b.part, cap * sizeof(double)));
    b.cap = cap;
  }
  *out = &b;
  return HYP_OK;
}

static hyp_status validate_jobs(const hyp_grad_job* jobs, int n, hyp_dtype* dt) {
  if (!jobs || n < 1 || n > kMaxJobs) return fail(HYP_ERR_ARG, "batched gradients: 1..16 jobs required");
  for (int j = 0; j < n; ++j) {
    const hyp_grad_job& g = jobs[j];
    if (!sector_of(g.sector) || !g.ops_dev || !g.psi_dev || !g.sigma_dev || !g.grad_dev || g.n_ops < 0)
      return fail(HYP_ERR_ARG, "batched gradients: NULL field or negative n_ops");
    if (g.dtype != jobs[0].dtype || (g.dtype != HYP_F64 && g.dtype != HYP_F32))
      return fail(HYP_ERR_ARG, "batched gradients: all jobs need one dtype (f64 or f32)");
  }
  *dt = jobs[0].dtype;
  // every excitation is checked on the host before any launch (the kernel
  // sizes its LDS lists for valid singles and doubles only)
  std::vector<hyp_exc> h;
  for (int j = 0; j < n; ++j) {
    if (jobs[j].n_ops == 0) continue;
    h.resize((size_t)jobs[j].n_ops);
    HYP_HIP(hipMemcpy(h.data(), jobs[j].ops_dev, sizeof(hyp_exc) * h.size(), hipMemcpyDeviceToHost));
    for (const hyp_exc& e : h) {
      hyp_status r = validate_exc(sector_of(jobs[j].sector), e);
      if (r != HYP_OK) return r;
    }
  }
  return HYP_OK;
}

static hyp_status launch_batched(const hyp_grad_job* jobs, int n, hyp_dtype dt,
                                 const hyp_sweep_tile& tile, hipStream_t st) {
  BatchArgs a{};
  SumArgs s{};
  a.n_jobs = s.n_jobs = n;
  a.nch = s.nch = tile.chunks;
  int64_t items = 0, parts = 0, gens = 0;
  for (int j = 0; j < n; ++j) {
    Sector* S = sector_of(jobs[j].sector);
    a.job[j].S = S->dev();
    a.job[j].ops = jobs[j].ops_dev;
    a.job[j].psi = jobs[j].psi_dev;
    a.job[j].sig = jobs[j].sigma_dev;
    a.job[j].n_ops = jobs[j].n_ops;
    a.job[j].item_off = items;
    a.job[j].part_off = parts;
    s.part_off[j] = parts;
    s.n_off[j] = gens;
    s.grad[j] = jobs[j].grad_dev;
    items += jobs[j].n_ops * tile.chunks;
    parts += jobs[j].n_ops * tile.chunks;
    gens += jobs[j].n_ops;
  }
  s.n_off[n] = gens;
  a.total = items;
  if (items == 0) return HYP_OK;
  BatchScratch* b = nullptr;
  hyp_status r = batch_scratch((size_t)parts, &b);
  if (r != HYP_OK) return r;
  a.counter = b->counter;
  a.part = b->part;
  s.part = b->part;
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  const int grid = std::max(1, g_cus[dev] * tile.blocks_per_cu);
  HYP_LAUNCH("k_reset_counter", k_reset_counter, dim3(1), dim3(64), 0, st, a.counter);
  if (dt == HYP_F64)
    HYP_LAUNCH("k_pool_grad_persistent", k_pool_grad_persistent<double>, dim3(grid), dim3(tile.threads), 0,
               st, a);
  else
    HYP_LAUNCH("k_pool_grad_persistent", k_pool_grad_persistent<float>, dim3(grid), dim3(tile.threads), 0,
               st, a);
  HYP_LAUNCH("k_sum_batched", k_sum_batched, dim3((unsigned)((gens + 255) / 256)), dim3(256), 0, st, s);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

static bool tile_ok(const hyp_sweep_tile& t) {
  return (t.threads == 64 || t.threads == 128 || t.threads == 256 || t.threads == 512 ||
          t.threads == 1024) &&
         t.chunks >= 1 && t.chunks <= 256 && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32;
}

}  // namespace hyp

using namespace hyp;

extern "C" {

hyp_status hyp_pool_gradients_batched(const hyp_grad_job* jobs, int n_jobs, const hyp_sweep_tile* tile,
                                      void* stream) {
  hyp_dtype dt;
  hyp_status r = validate_jobs(jobs, n_jobs, &dt);
  if (r != HYP_OK) return r;
  hyp_sweep_tile t = tile ? *tile : hyp_sweep_tile{256, 16, 4, 0};
  if (!tile_ok(t)) return fail(HYP_ERR_ARG, "batched gradients: bad tile");
  hipStream_t st = (hipStream_t)stream;
  // full pools: the transition-value sweep per instance; subsets: one fused launch
  std::vector<hyp_grad_job> rest;
  for (int i = 0; i < n_jobs; ++i) {
    Sector* S = sector_of(jobs[i].sector);
    if (prefer_full_sweep(S, jobs[i].n_ops)) {
      r = launch_pool_gradients(S, dt, jobs[i].ops_dev, jobs[i].n_ops, jobs[i].psi_dev, jobs[i].sigma_dev,
                                jobs[i].grad_dev, st);
      if (r != HYP_OK) return r;
    } else {
      rest.push_back(jobs[i]);
    }
  }
  if (rest.empty()) return HYP_OK;
  return launch_batched(rest.data(), (int)rest.size(), dt, t, st);
}

hyp_status hyp_tune_pool_gradients(const hyp_grad_job* jobs, int n_jobs, int reps,
                                   hyp_sweep_tile* best, double* best_ms, void* stream) {
  hyp_dtype dt;
  hyp_status r = validate_jobs(jobs, n_jobs, &dt);
  if (r != HYP_OK) return r;
  if (!best || !best_ms || reps < 1) return fail(HYP_ERR_ARG, "hyp_tune_pool_gradients: bad output or reps");
  hipStream_t st = (hipStream_t)stream;
  static const int th[] = {128, 256, 512};
  static const int ch[] = {4, 8, 16, 32};
  static const int bp[] = {2, 4, 8};
  hipEvent_t e0, e1;
  HYP_HIP(hipEventCreate(&e0));
  HYP_HIP(hipEventCreate(&e1));
  double bms = 1e300;
  hyp_sweep_tile bt{256, 16, 4, 0};
  for (int a : th)
    for (int c : ch)
      for (int b : bp) {
        hyp_sweep_tile t{a, c, b, 0};
        r = launch_batched(jobs, n_jobs, dt, t, st);  // warm-up, grows scratch
        if (r != HYP_OK) break;
        HYP_HIP(hipStreamSynchronize(st));
        HYP_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < reps && r == HYP_OK; ++i) r = launch_batched(jobs, n_jobs, dt, t, st);
        HYP_HIP(hipEventRecord(e1, st));
        HYP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        HYP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r == HYP_OK && ms / reps < bms) {
          bms = ms / reps;
          bt = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != HYP_OK) return r;
  *best = bt;
  *best_ms = bms;
  return HYP_OK;
}

}  // extern "C"
