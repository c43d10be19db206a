// Paired-determinant kernels: ADAPT-VQE pool gradients g_k = 2 <sigma|A_k psi>
// ("Numerical performance": the gradient over the operator pool is the
// bottleneck that selects each new operator), the exponentiated fermionic
// operator exp(theta A) psi ("Sparse State-Vector Emulation"), and the fused
// adjoint step of the inner optimiser.
//
// A generator A = tau - tau^dagger splits into an alpha part and a beta part
// (each an identity, a single or a double in one spin).  Its pairs
// (D, D' = tau D) are the product of the qualifying alpha strings and the
// qualifying beta strings, and the sign factorises: s = s_alpha * s_beta,
// each the sign of applying that spin's ladder operators (annihilators
// ascending, then creators descending) to that spin's string.  Pairs of one
// generator are disjoint, so rotations are in place and race-free.
#include "hyp_internal.h"

#include <cmath>
#include <vector>

namespace hyp {

constexpr int kListMax = 3432;  // max C(M-2, N-1) for M <= 16
constexpr int kPairChunks = 16; // beta-entry chunks per generator (gradient partials)
constexpr int kPairThreads = 256;

__constant__ int c_binom[17][17];

struct SpinPart {
  uint32_t cm, am;   // creation / annihilation orbitals of this spin (orbital coords)
  int count;         // number of qualifying strings
  int nsel, nfree;   // electrons to place among the free orbitals
  uint32_t free;
};

__device__ inline SpinPart make_part(uint32_t cm, uint32_t am, int M, int N) {
  SpinPart p;
  p.cm = cm;
  p.am = am;
  p.free = ~(cm | am) & ((1u << M) - 1u);
  p.nfree = __popc(p.free);
  p.nsel = N - __popc(am);
  p.count = (p.nsel < 0 || p.nsel > p.nfree) ? 0 : c_binom[p.nfree][p.nsel];
  return p;
}

// i-th qualifying string (colex order of the free-orbital subset)
__device__ inline uint32_t part_string(const SpinPart& p, int i) {
  uint32_t pos = 0;  // subset of {0..nfree-1}
  int r = i;
  for (int j = p.nsel; j >= 1; --j) {
    int c = j - 1;
    while (c + 1 < p.nfree && c_binom[c + 1][j] <= r) ++c;
    r -= c_binom[c][j];
    pos |= 1u << c;
  }
  // scatter subset positions onto the free orbitals
  uint32_t s = p.am, f = p.free;
  for (int b = 0; f; ++b) {
    uint32_t low = f & (~f + 1u);
    if (pos & (1u << b)) s |= low;
    f ^= low;
  }
  return s;
}

// sign of applying this spin's part of tau to string s: annihilators in
// ascending orbital order, then creators in descending order
__device__ inline int part_sign(uint32_t cm, uint32_t am, uint32_t s) {
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

__device__ inline int rank_of(const RankTables* t, uint32_t s) {
  return t->lo[s & 255u] + t->hi[(s >> 8) & 255u];
}

struct PairCtx {
  SpinPart pa, pb;
  bool a_id;  // alpha part is the identity
};

__device__ inline PairCtx make_ctx(hyp_exc op, const SectorDev& S) {
  const uint32_t m = (1u << S.M) - 1u;
  PairCtx c;
  c.pa = make_part(op.cre & m, op.ann & m, S.M, S.na);
  c.pb = make_part((op.cre >> S.M) & m, (op.ann >> S.M) & m, S.M, S.nb);
  c.a_id = (c.pa.cm | c.pa.am) == 0;
  return c;
}

// Build the alpha list (rank J | rank I << 14 | sign << 28) in LDS.
__device__ inline void build_alpha_list(const PairCtx& c, const SectorDev& S, uint32_t* lst) {
  if (c.a_id) return;
  for (int i = threadIdx.x; i < c.pa.count; i += blockDim.x) {
    uint32_t J = part_string(c.pa, i);
    uint32_t I = J ^ c.pa.am ^ c.pa.cm;
    int sg = part_sign(c.pa.cm, c.pa.am, J) & S.fsign;
    lst[i] = (uint32_t)rank_of(S.arank, J) | ((uint32_t)rank_of(S.arank, I) << 14) | ((uint32_t)sg << 28);
  }
}

template <typename T>
__device__ inline double ld(const T* p, int64_t i) {
  return (double)p[i];
}

// ---------------------------------------------------------------- gradients

template <typename T>
__global__ void __launch_bounds__(kPairThreads) k_pool_grad(SectorDev S, const hyp_exc* ops,
                                                           const T* psi, const T* sig,
                                                           const uint32_t* __restrict__ nzb,
                                                           const uint32_t* __restrict__ nza,
                                                           double* part, int* bad_rec) {
  __shared__ uint32_t lst[kListMax];
  __shared__ double red[kPairThreads / 64];
  const int k = blockIdx.x, chunk = blockIdx.y;
  const int bad = exc_status(ops[k], S.M);
  if (bad != HYP_OK) {  // an invalid excitation: its gradient is NaN, nothing is indexed
    if (threadIdx.x == 0) {
      part[(int64_t)k * kPairChunks + chunk] = __builtin_nan("");
      if (chunk == 0) note_bad_exc(bad_rec, bad, k);
    }
    return;
  }
  const PairCtx c = make_ctx(ops[k], S);
  build_alpha_list(c, S, lst);
  __syncthreads();
  const int nA = c.a_id ? S.da : c.pa.count;
  const int nB = c.pb.count;
  const bool b_id = (c.pb.cm | c.pb.am) == 0;
  const int b0 = (int)((int64_t)nB * chunk / kPairChunks), b1 = (int)((int64_t)nB * (chunk + 1) / kPairChunks);
  double acc = 0.0;
  for (int jb = b0; jb < b1; ++jb) {
    int rJb, rIb, sb;
    if (b_id) {
      rJb = rIb = jb;
      sb = 0;
    } else {
      uint32_t Jb = part_string(c.pb, jb);
      uint32_t Ib = Jb ^ c.pb.am ^ c.pb.cm;
      rJb = rank_of(S.brank, Jb);
      rIb = rank_of(S.brank, Ib);
      sb = part_sign(c.pb.cm, c.pb.am, Jb) & S.fsign;
    }
    // support skipping: a pair contributes only if psi[D] or psi[D'] can be
    // nonzero (its beta row and alpha column both in psi's support)
    const bool zJ = !nzb || nzb[rJb], zI = !nzb || nzb[rIb];
    if (!zJ && !zI) continue;
    const int64_t oJ = (int64_t)rJb * S.da, oI = (int64_t)rIb * S.da;
    double rs = 0.0;
    for (int t = threadIdx.x; t < nA; t += blockDim.x) {
      int rJa, rIa, sa;
      if (c.a_id) {
        rJa = rIa = t;
        sa = 0;
      } else {
        uint32_t e = lst[t];
        rJa = e & 0x3fff;
        rIa = (e >> 14) & 0x3fff;
        sa = (e >> 28) & 1;
      }
      if (nza && !((zJ && nza[rJa]) || (zI && nza[rIa]))) continue;
      const int64_t D = oJ + rJa, Dp = oI + rIa;
      // sigma[D'] psi[D] - sigma[D] psi[D'] (FP32 storage: FP32 products)
      double v;
      if (sizeof(T) == 4)
        v = (double)((float)sig[Dp] * (float)psi[D]) - (double)((float)sig[D] * (float)psi[Dp]);
      else
        v = ld(sig, Dp) * ld(psi, D) - ld(sig, D) * ld(psi, Dp);
      rs += (sa ? -v : v);
    }
    acc += sb ? -rs : rs;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kPairThreads / 64; ++w) s += red[w];
    part[(int64_t)k * kPairChunks + chunk] = s;
  }
}

__global__ void k_sum_chunks(const double* part, int64_t n, double scale, double* out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int c = 0; c < kPairChunks; ++c) s += part[k * kPairChunks + c];
  out[k] = scale * s;
}

// ---------------------------------------------------------------- rotation

// theta_dev != nullptr: the angle is read from device memory (graph replay
// with new parameters); otherwise (co, sn) are used.
template <typename T>
__global__ void __launch_bounds__(kPairThreads) k_rotate(SectorDev S, hyp_exc op, double co,
                                                        double sn, const double* theta_dev,
                                                        T* psi, int nchunk) {
  __shared__ uint32_t lst[kListMax];
  const PairCtx c = make_ctx(op, S);
  build_alpha_list(c, S, lst);
  if (theta_dev) {
    co = cos(*theta_dev);
    sn = sin(*theta_dev);
  }
  __syncthreads();
  const int nA = c.a_id ? S.da : c.pa.count;
  const int nB = c.pb.count;
  const bool b_id = (c.pb.cm | c.pb.am) == 0;
  const int chunk = blockIdx.x;
  const int b0 = (int)((int64_t)nB * chunk / nchunk), b1 = (int)((int64_t)nB * (chunk + 1) / nchunk);
  for (int jb = b0; jb < b1; ++jb) {
    int rJb, rIb, sb;
    if (b_id) {
      rJb = rIb = jb;
      sb = 0;
    } else {
      uint32_t Jb = part_string(c.pb, jb);
      uint32_t Ib = Jb ^ c.pb.am ^ c.pb.cm;
      rJb = rank_of(S.brank, Jb);
      rIb = rank_of(S.brank, Ib);
      sb = part_sign(c.pb.cm, c.pb.am, Jb) & S.fsign;
    }
    const int64_t oJ = (int64_t)rJb * S.da, oI = (int64_t)rIb * S.da;
    for (int t = threadIdx.x; t < nA; t += blockDim.x) {
      int rJa, rIa, sa;
      if (c.a_id) {
        rJa = rIa = t;
        sa = 0;
      } else {
        uint32_t e = lst[t];
        rJa = e & 0x3fff;
        rIa = (e >> 14) & 0x3fff;
        sa = (e >> 28) & 1;
      }
      const int64_t D = oJ + rJa, Dp = oI + rIa;
      const double s = ((sa ^ sb) & 1) ? -sn : sn;
      const double x0 = (double)psi[D], x1 = (double)psi[Dp];
      psi[D] = (T)(co * x0 - s * x1);
      psi[Dp] = (T)(s * x0 + co * x1);
    }
  }
}

// ---------------------------------------------------------------- adjoint step

// part[chunk] = sum over pairs of s (lam[D'] phi[D] - lam[D] phi[D']) with the
// pre-rotation values, then phi <- exp(-theta A) phi, lam <- exp(-theta A) lam
template <typename T>
__global__ void __launch_bounds__(kPairThreads) k_adjoint_step(SectorDev S, hyp_exc op,
                                                              const double* theta, T* phi,
                                                              T* lam, double* part, int nchunk) {
  __shared__ uint32_t lst[kListMax];
  __shared__ double red[kPairThreads / 64];
  const PairCtx c = make_ctx(op, S);
  build_alpha_list(c, S, lst);
  __syncthreads();
  const double th = -theta[0];
  const double co = cos(th), sn = sin(th);
  const int nA = c.a_id ? S.da : c.pa.count;
  const int nB = c.pb.count;
  const bool b_id = (c.pb.cm | c.pb.am) == 0;
  const int chunk = blockIdx.x;
  const int b0 = (int)((int64_t)nB * chunk / nchunk), b1 = (int)((int64_t)nB * (chunk + 1) / nchunk);
  double acc = 0.0;
  for (int jb = b0; jb < b1; ++jb) {
    int rJb, rIb, sb;
    if (b_id) {
      rJb = rIb = jb;
      sb = 0;
    } else {
      uint32_t Jb = part_string(c.pb, jb);
      uint32_t Ib = Jb ^ c.pb.am ^ c.pb.cm;
      rJb = rank_of(S.brank, Jb);
      rIb = rank_of(S.brank, Ib);
      sb = part_sign(c.pb.cm, c.pb.am, Jb) & S.fsign;
    }
    const int64_t oJ = (int64_t)rJb * S.da, oI = (int64_t)rIb * S.da;
    for (int t = threadIdx.x; t < nA; t += blockDim.x) {
      int rJa, rIa, sa;
      if (c.a_id) {
        rJa = rIa = t;
        sa = 0;
      } else {
        uint32_t e = lst[t];
        rJa = e & 0x3fff;
        rIa = (e >> 14) & 0x3fff;
        sa = (e >> 28) & 1;
      }
      const int64_t D = oJ + rJa, Dp = oI + rIa;
      const int neg = (sa ^ sb) & 1;
      const double f0 = (double)phi[D], f1 = (double)phi[Dp];
      const double l0 = (double)lam[D], l1 = (double)lam[Dp];
      const double v = l1 * f0 - l0 * f1;
      acc += neg ? -v : v;
      const double s = neg ? -sn : sn;
      phi[D] = (T)(co * f0 - s * f1);
      phi[Dp] = (T)(s * f0 + co * f1);
      lam[D] = (T)(co * l0 - s * l1);
      lam[Dp] = (T)(s * l0 + co * l1);
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kPairThreads / 64; ++w) s += red[w];
    part[chunk] = s;
  }
}

__global__ void k_sum_n(const double* part, int n, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = scale * s;
  }
}

// ---------------------------------------------------------------- host side

static bool g_binom_ready[64];

hyp_status ensure_binom() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  if (g_binom_ready[dev]) return HYP_OK;
  int tab[17][17];
  for (int m = 0; m <= 16; ++m)
    for (int k = 0; k <= 16; ++k) {
      int64_t r = 0;
      if (k <= m) {
        r = 1;
        for (int i = 1; i <= k; ++i) r = r * (m - k + i) / i;
      }
      tab[m][k] = (int)r;
    }
  HYP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), tab, sizeof(tab)));
  g_binom_ready[dev] = true;
  return HYP_OK;
}

hyp_status validate_exc(const Sector* S, hyp_exc op) {
  const int n = 2 * S->M;
  const uint32_t all = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
  const uint32_t m = (1u << S->M) - 1u;
  if ((op.cre | op.ann) & ~all) return fail(HYP_ERR_ARG, "excitation mask bit >= 2*n_orb");
  const int nc = __builtin_popcount(op.cre), na = __builtin_popcount(op.ann);
  if (nc != na || nc < 1 || nc > 2) return fail(HYP_ERR_ARG, "excitation needs |cre| == |ann| in {1, 2}");
  if (op.cre & op.ann) return fail(HYP_ERR_ARG, "excitation cre and ann overlap");
  if (__builtin_popcount(op.cre & m) != __builtin_popcount(op.ann & m))
    return fail(HYP_ERR_SECTOR, "excitation changes N_alpha / N_beta");
  return HYP_OK;
}

// [0] the largest status met, [1] the smallest list position with it
// (positions of one call; cleared by hyp_pool_check)
__device__ int g_bad_exc[2] = {0, 0x7fffffff};

int* bad_exc_record() {
  static int* rec[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!rec[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_bad_exc)) != hipSuccess) return nullptr;
    rec[dev] = (int*)p;
  }
  return rec[dev];
}

// grow-only per-sector scratch for chunk partials
hyp_status pair_scratch(Sector* S, size_t n_doubles, double** out);

template <typename T>
static hyp_status launch_pool_grad(Sector* S, const hyp_exc* ops, int64_t n_ops, const void* psi,
                                   const void* sig, double* grad, hipStream_t st) {
  double* part = nullptr;
  hyp_status r = pair_scratch(S, (size_t)n_ops * kPairChunks, &part);
  if (r != HYP_OK) return r;
  const uint32_t* nz = nullptr;
  if (support_skip()) {
    r = support_flags(S, sizeof(T) == 4 ? HYP_F32 : HYP_F64, psi, &nz, st);
    if (r != HYP_OK) return r;
  }
  int* rec = bad_exc_record();
  if (!rec) return fail(HYP_ERR_HIP, "excitation check record not found");
  // grid.x is limited to 2^31-1, n_ops <= 2^24 here
  HYP_LAUNCH("k_pool_grad", k_pool_grad<T>, dim3((unsigned)n_ops, kPairChunks), dim3(kPairThreads), 0, st,
             S->dev(), ops, (const T*)psi, (const T*)sig, nz, nz ? nz + S->db : nullptr, part, rec);
  HYP_LAUNCH("k_sum_chunks", k_sum_chunks, dim3((unsigned)((n_ops + 255) / 256)), dim3(256), 0, st, part,
             n_ops, 2.0, grad);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

static int g_sweep_mode = 0;  // 0 automatic, 1 pairs, 2 transition values, 3 per-stage bins
static int g_pool_kind = 0;   // 0 fermionic excitations, 1 qubit excitations

int pool_kind() { return g_pool_kind; }

static int64_t full_pool_size(int M) {
  auto C = [](int64_t m, int64_t k) {
    if (k < 0 || k > m) return (int64_t)0;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) r = r * (m - k + i) / i;
    return r;
  };
  return 2 * C(M, 2) + 6 * C(M, 4) + (int64_t)(M * (M - 1)) * (M * (M - 1)) / 2;
}

hyp_status launch_pool_gradients(Sector* S, hyp_dtype dt, const hyp_exc* ops, int64_t n_ops,
                                 const void* psi, const void* sig, double* grad, hipStream_t st) {
  hyp_status r = ensure_binom();
  if (r != HYP_OK) return r;
  if (n_ops == 0) return HYP_OK;
  // the transition-value sweep costs about one mixed H psi pass whatever the
  // list; it pays when the list covers a good part of the pool
  const bool big = n_ops * 4 >= full_pool_size(S->M);
  if (g_sweep_mode == 2 || (g_sweep_mode == 0 && big))
    return launch_tdens(S, dt, ops, n_ops, psi, sig, grad, st, false);
  if (g_sweep_mode == 3) {
    if (tdens_bytes(S) > ((size_t)40 << 30))
      return fail(HYP_ERR_ARG, "hyp_pool_gradients: per-stage bin scratch above 40 GiB for this sector");
    return launch_tdens(S, dt, ops, n_ops, psi, sig, grad, st, true);
  }
  if (dt == HYP_F64) return launch_pool_grad<double>(S, ops, n_ops, psi, sig, grad, st);
  return launch_pool_grad<float>(S, ops, n_ops, psi, sig, grad, st);
}

bool prefer_full_sweep(const Sector* S, int64_t n_ops) {
  return g_sweep_mode != 1 && n_ops * 4 >= full_pool_size(S->M);
}

hyp_status set_sweep_mode(int mode) {
  if (mode < 0 || mode > 3) return fail(HYP_ERR_ARG, "hyp_set_sweep_mode: mode must be 0, 1, 2 or 3");
  g_sweep_mode = mode;
  return HYP_OK;
}

static int rot_chunks(const Sector* S, hyp_exc op) {
  // number of beta entries of the generator bounds the useful chunk count
  const uint32_t m = (1u << S->M) - 1u;
  int cb = __builtin_popcount((op.cre >> S->M) & m);
  int64_t nb = S->db;
  if (cb) {
    int nfree = S->M - 2 * cb;
    int nsel = S->nb - cb;
    int64_t r = 1;
    if (nsel < 0 || nsel > nfree) return 1;
    for (int i = 1; i <= nsel; ++i) r = r * (nfree - nsel + i) / i;
    nb = r;
  }
  int64_t ch = std::min<int64_t>(nb, 2048);
  return (int)std::max<int64_t>(ch, 1);
}

hyp_status launch_rotate(Sector* S, hyp_dtype dt, hyp_exc op, double theta, const double* theta_dev,
                         void* psi, hipStream_t st) {
  hyp_status r = ensure_binom();
  if (r != HYP_OK) return r;
  int nch = rot_chunks(S, op);
  double co = std::cos(theta), sn = std::sin(theta);
  if (dt == HYP_F64)
    HYP_LAUNCH("k_rotate", k_rotate<double>, dim3(nch), dim3(kPairThreads), 0, st, S->dev(), op, co, sn,
               theta_dev, (double*)psi, nch);
  else
    HYP_LAUNCH("k_rotate", k_rotate<float>, dim3(nch), dim3(kPairThreads), 0, st, S->dev(), op, co, sn,
               theta_dev, (float*)psi, nch);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

// theta and grad_out are device pointers (graph-capturable); part has room
// for rot_chunks doubles.
hyp_status launch_adjoint_step(Sector* S, hyp_dtype dt, hyp_exc op, const double* theta_dev,
                               void* phi, void* lam, double* part, double* grad_out,
                               hipStream_t st) {
  int nch = rot_chunks(S, op);
  if (dt == HYP_F64)
    HYP_LAUNCH("k_adjoint_step", k_adjoint_step<double>, dim3(nch), dim3(kPairThreads), 0, st, S->dev(), op,
                       theta_dev, (double*)phi, (double*)lam, part, nch);
  else
    HYP_LAUNCH("k_adjoint_step", k_adjoint_step<float>, dim3(nch), dim3(kPairThreads), 0, st, S->dev(), op,
                       theta_dev, (float*)phi, (float*)lam, part, nch);
  HYP_LAUNCH("k_sum_n", k_sum_n, dim3(1), dim3(64), 0, st, part, nch, 2.0, grad_out);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

int max_rot_chunks() { return 2048; }

}  // namespace hyp

using namespace hyp;

extern "C" {

hyp_status hyp_set_sweep_mode(int mode) { return set_sweep_mode(mode); }

hyp_status hyp_set_pool_kind(int kind) {
  if (kind != 0 && kind != 1) return fail(HYP_ERR_ARG, "hyp_set_pool_kind: kind must be 0 or 1");
  g_pool_kind = kind;
  return HYP_OK;
}

hyp_status hyp_pool_gradients(hyp_sector sh, hyp_dtype dtype, const hyp_exc* ops, int64_t n_ops,
                              const void* psi, const void* sigma, double* grad, void* stream) {
  Sector* S = sector_of(sh);
  if (!S || !ops || !psi || !sigma || !grad) return fail(HYP_ERR_ARG, "hyp_pool_gradients: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_pool_gradients: bad dtype");
  if (n_ops < 0 || n_ops > (int64_t)1 << 24) return fail(HYP_ERR_ARG, "hyp_pool_gradients: n_ops out of range");
  if (n_ops == 0) return HYP_OK;
  // the list is in device memory: every kernel that reads an excitation
  // checks it there (an invalid one gets a NaN gradient and is recorded for
  // hyp_pool_check), so nothing here waits for the device
  return launch_pool_gradients(S, dtype, ops, n_ops, psi, sigma, grad, (hipStream_t)stream);
}

// Scratch of hyp_pool_gradients_noalloc: the pair kernel's per-chunk
// partials, one array per GPU for the life of the process, shared by every
// call on that GPU (overlapping calls race).  Host code uses only the device
// address taken with hipGetSymbolAddress, never the array's name.
constexpr int64_t kNoAllocOps = 32768;
static __device__ __align__(256) double scratch[kNoAllocOps * kPairChunks];
static double* g_scratch_ptr[64] = {};

hyp_status hyp_pool_gradients_noalloc(hyp_sector sh, hyp_dtype dtype, const hyp_exc* ops, int64_t n_ops,
                                      const void* psi, const void* sigma, double* grad, void* stream) {
  Sector* S = sector_of(sh);
  if (!S || !ops || !psi || !sigma || !grad) return fail(HYP_ERR_ARG, "hyp_pool_gradients_noalloc: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_pool_gradients_noalloc: bad dtype");
  if (n_ops < 0 || n_ops > kNoAllocOps)
    return fail(HYP_ERR_ARG, "hyp_pool_gradients_noalloc: n_ops must be in [0, " + std::to_string(kNoAllocOps) +
                                 "] (the size of its static scratch)");
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    // set-up, once per device with that device current: the array's
    // address on this GPU, and the binomial table of the pair kernel
    void* p = nullptr;
    HYP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    hyp_status r = ensure_binom();
    if (r != HYP_OK) return r;
    g_scratch_ptr[dev] = (double*)p;
  }
  if (n_ops == 0) return HYP_OK;
  int* rec = bad_exc_record();
  if (!rec) return fail(HYP_ERR_HIP, "excitation check record not found");
  hipStream_t st = (hipStream_t)stream;
  double* part = g_scratch_ptr[dev];  // every (generator, chunk) partial is written before it is read
  if (dtype == HYP_F64)
    HYP_LAUNCH("k_pool_grad", k_pool_grad<double>, dim3((unsigned)n_ops, kPairChunks), dim3(kPairThreads), 0, st,
               S->dev(), ops, (const double*)psi, (const double*)sigma, nullptr, nullptr, part, rec);
  else
    HYP_LAUNCH("k_pool_grad", k_pool_grad<float>, dim3((unsigned)n_ops, kPairChunks), dim3(kPairThreads), 0, st,
               S->dev(), ops, (const float*)psi, (const float*)sigma, nullptr, nullptr, part, rec);
  HYP_LAUNCH("k_sum_chunks", k_sum_chunks, dim3((unsigned)((n_ops + 255) / 256)), dim3(256), 0, st, part, n_ops,
             2.0, grad);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_pool_check(void* stream) {
  hipStream_t st = (hipStream_t)stream;
  int* rec = bad_exc_record();
  if (!rec) return fail(HYP_ERR_HIP, "hyp_pool_check: record not found");
  int h[2] = {0, 0x7fffffff};
  HYP_HIP(hipMemcpyAsync(h, rec, sizeof(h), hipMemcpyDeviceToHost, st));
  HYP_HIP(hipStreamSynchronize(st));
  if (h[0] == HYP_OK) return HYP_OK;
  const int clear[2] = {0, 0x7fffffff};
  HYP_HIP(hipMemcpy(rec, clear, sizeof(clear), hipMemcpyHostToDevice));
  const std::string what = h[0] == HYP_ERR_SECTOR ? "changes N_alpha / N_beta"
                                                  : "is not a valid excitation (mask bits, counts or overlap)";
  return fail((hyp_status)h[0], "hyp_pool_gradients: excitation " + std::to_string(h[1]) + " " + what);
}

hyp_status hyp_apply_excitation(hyp_sector sh, hyp_dtype dtype, hyp_exc op, double theta,
                                void* psi, void* stream) {
  Sector* S = sector_of(sh);
  if (!S || !psi) return fail(HYP_ERR_ARG, "hyp_apply_excitation: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_apply_excitation: bad dtype");
  if (!std::isfinite(theta)) return fail(HYP_ERR_ARG, "hyp_apply_excitation: non-finite theta");
  hyp_status r = validate_exc(S, op);
  if (r != HYP_OK) return r;
  return launch_rotate(S, dtype, op, theta, nullptr, psi, (hipStream_t)stream);
}

hyp_status hyp_apply_excitations(hyp_sector sh, hyp_dtype dtype, const hyp_exc* ops, const double* theta,
                                 int64_t n, void* psi, void* stream) {
  Sector* S = sector_of(sh);
  if (!S || !psi || n < 0 || (n > 0 && (!ops || !theta)))
    return fail(HYP_ERR_ARG, "hyp_apply_excitations: NULL argument or negative count");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_apply_excitations: bad dtype");
  // everything is validated before the first rotation is enqueued
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(theta[i])) return fail(HYP_ERR_ARG, "hyp_apply_excitations: non-finite theta");
    hyp_status r = validate_exc(S, ops[i]);
    if (r != HYP_OK) return r;
  }
  for (int64_t i = 0; i < n; ++i) {
    hyp_status r = launch_rotate(S, dtype, ops[i], theta[i], nullptr, psi, (hipStream_t)stream);
    if (r != HYP_OK) return r;
  }
  return HYP_OK;
}

}  // extern "C"
