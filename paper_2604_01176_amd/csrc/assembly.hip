// Device-side Hamiltonian assembly: molecular integrals -> Jordan-Wigner
// Pauli list, merged and sorted by (x, z) on the GPU (paper, "Sparse
// State-Vector Emulation": the Hamiltonian is assembled on the GPU by summing
// the contributions of the individual fermionic operators after mapping them
// to qubits; there into a CSR matrix, here into the X-grouped Pauli table the
// matrix-free kernels consume).
//
// Conventions (the same as hyp_build_hamiltonian's input): spin orbital
// P = p + s M on qubit P (blocked spin order), P(x, z) the Pauli string with
// Y where both bits are set, and
//   H = e_core + sum_{pq s} h_pq a+_{ps} a_{qs}
//     + 1/2 sum_{pqrs, s t} g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs}   (chemist's notation).
// Under Jordan-Wigner a_P = Z_0..Z_{P-1} (X_P + i Y_P) / 2 and
// a+_P = Z_0..Z_{P-1} (X_P - i Y_P) / 2, so a product of k ladder operators is
// a sum of 2^k Pauli strings, each picking the X part (P(e, m), factor 1/2)
// or the Y part (P(e, m|e), factor +-i/2) of every operator (e = 2^P,
// m = 2^P - 1).  Writing P(x, z) = i^{|x&z|} X^x Z^z, the product of two strings is
// P(x1,z1) P(x2,z2) = i^k P(x1^x2, z1^z2),
// k = |x1&z1| + |x2&z2| + 2|z1&x2| - |(x1^x2)&(z1^z2)|  (mod 4).
//
// Pipeline: one thread per (fermionic term, choice of parts) writes its key
// (x << 32 | z) and complex coefficient; a stable radix sort by key (rocPRIM
// through hipCUB) brings equal strings together in generation order; one
// thread per run of equal keys sums the run in double-double arithmetic
// (error-free two-sums), so the merged coefficient is the correctly rounded
// sum in all but near-tie cases, and sums of exactly cancelling
// contributions come out at the level of 1e-30 of their terms; such
// residues (below 1e-14 of the run's sum of magnitudes) are exact zeros and
// dropped.  An imaginary part above that level means the integrals do not
// define a real Hamiltonian (HYP_ERR_NONREAL).
#include "hyp_internal.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

namespace hyp {

namespace {

constexpr uint64_t kNoTerm = ~0ull;  // key of a slot that carries no term (sorts last)

__device__ inline int popc32(uint32_t v) { return __popc(v); }

// Slots: one-body (s, p, q) x 4 choices, then two-body (p, q, r, u, s, t) x 16
// choices, then one slot for e_core.
__global__ void k_jw_expand(int M, const double* __restrict__ h, const double* __restrict__ g, double e_core,
                            int64_t n1, int64_t n2, uint64_t* __restrict__ key, int* __restrict__ idx,
                            double* __restrict__ re, double* __restrict__ im) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = n1 + n2 + 1;
  if (i >= n) return;
  idx[i] = (int)i;
  int nops = 0;
  int q[4];
  bool dag[4];
  double v = 0.0;
  int choice = 0;
  if (i < n1) {
    choice = (int)(i & 3);
    const int64_t t = i >> 2;
    const int qq = (int)(t % M), p = (int)((t / M) % M), s = (int)(t / ((int64_t)M * M));
    v = h[p * M + qq];
    nops = 2;
    q[0] = p + s * M; dag[0] = true;
    q[1] = qq + s * M; dag[1] = false;
  } else if (i < n1 + n2) {
    const int64_t j = i - n1;
    choice = (int)(j & 15);
    int64_t t = j >> 4;
    const int tt = (int)(t & 1); t >>= 1;
    const int s = (int)(t & 1); t >>= 1;
    const int u = (int)(t % M); t /= M;
    const int r = (int)(t % M); t /= M;
    const int qq = (int)(t % M); t /= M;
    const int p = (int)t;
    const int P = p + s * M, Q = qq + s * M, R = r + tt * M, U = u + tt * M;
    if (P != R && Q != U) v = 0.5 * g[(((int64_t)p * M + qq) * M + r) * M + u];
    nops = 4;
    q[0] = P; dag[0] = true;
    q[1] = R; dag[1] = true;
    q[2] = U; dag[2] = false;
    q[3] = Q; dag[3] = false;
  } else {
    v = e_core;  // identity
  }
  if (v == 0.0) {
    key[i] = kNoTerm;
    re[i] = 0.0;
    im[i] = 0.0;
    return;
  }
  uint32_t x = 0u, z = 0u;
  int ipow = 0;  // power of i
  double mag = v;
  for (int k = 0; k < nops; ++k) {
    const uint32_t e = 1u << q[k], m = e - 1u;
    uint32_t x2 = e, z2 = m;
    if ((choice >> k) & 1) {
      z2 = m | e;
      ipow += dag[k] ? 3 : 1;  // -i/2 for a creator, +i/2 for an annihilator
    }
    mag *= 0.5;
    ipow += popc32(x & z) + popc32(x2 & z2) + 2 * popc32(z & x2) - popc32((x ^ x2) & (z ^ z2));
    x ^= x2;
    z ^= z2;
  }
  ipow &= 3;
  key[i] = ((uint64_t)x << 32) | z;
  re[i] = ipow == 0 ? mag : (ipow == 2 ? -mag : 0.0);
  im[i] = ipow == 1 ? mag : (ipow == 3 ? -mag : 0.0);
}

// head[i] = 1 where a run of equal keys starts (terms only)
__global__ void k_run_heads(const uint64_t* __restrict__ key, int64_t n, int* __restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  head[i] = (key[i] != kNoTerm && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

__device__ inline void two_sum(double a, double b, double* s, double* e) {
  const double t = a + b;
  const double bb = t - a;
  *e = (a - (t - bb)) + (b - bb);
  *s = t;
}

// One thread per sorted position that starts a run: the run's double-double
// sum of real and imaginary parts; keep[r] = 1 for a nonzero real sum.
__global__ void k_run_sums(const uint64_t* __restrict__ key, const int* __restrict__ idx, const double* __restrict__ re,
                           const double* __restrict__ im, const int* __restrict__ head, const int* __restrict__ rid,
                           int64_t n, uint64_t* __restrict__ rkey, double* __restrict__ rc, int* __restrict__ keep,
                           int* __restrict__ nonreal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  const uint64_t k = key[i];
  double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0, ar = 0.0, ai = 0.0;
  for (int64_t j = i; j < n && key[j] == k; ++j) {
    const int src = idx[j];
    double t;
    two_sum(sr, re[src], &sr, &t);
    er += t;
    two_sum(si, im[src], &si, &t);
    ei += t;
    ar += fabs(re[src]);
    ai += fabs(im[src]);
  }
  const double cr = sr + er, ci = si + ei;
  const int r = rid[i];
  rkey[r] = k;
  const bool zr = fabs(cr) <= 1e-14 * ar;
  rc[r] = zr ? 0.0 : cr;
  keep[r] = zr ? 0 : 1;
  if (!(fabs(ci) <= 1e-14 * ai)) atomicOr(nonreal, 1);
}

__global__ void k_emit(const uint64_t* __restrict__ rkey, const double* __restrict__ rc, const int* __restrict__ keep,
                       const int* __restrict__ pos, int64_t nrun, uint32_t* __restrict__ xo, uint32_t* __restrict__ zo,
                       double* __restrict__ co, int64_t cap) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrun || !keep[r]) return;
  const int64_t o = pos[r];
  if (o >= cap) return;
  xo[o] = (uint32_t)(rkey[r] >> 32);
  zo[o] = (uint32_t)(rkey[r] & 0xffffffffu);
  co[o] = rc[r];
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(1, n) * sizeof(T)); }
};

}  // namespace

// Assemble into device arrays; *n_out = number of terms (written up to cap).
hyp_status assemble_pauli(int M, const double* h, const double* g, double e_core, uint32_t* xo, uint32_t* zo,
                          double* co, int64_t cap, int64_t* n_out, hipStream_t st) {
  const int64_t n1 = (int64_t)2 * M * M * 4;
  const int64_t n2 = (int64_t)M * M * M * M * 4 * 16;
  const int64_t n = n1 + n2 + 1;
  if (n >= (int64_t)1 << 31) return fail(HYP_ERR_ARG, "hyp_assemble_pauli: too many terms");
  DevBuf<uint64_t> key, key2, rkey;
  DevBuf<int> idx, idx2, head, rid, keep, pos, flag;
  DevBuf<double> re, im, rc;
  HYP_HIP(key.alloc(n));
  HYP_HIP(key2.alloc(n));
  HYP_HIP(idx.alloc(n));
  HYP_HIP(idx2.alloc(n));
  HYP_HIP(re.alloc(n));
  HYP_HIP(im.alloc(n));
  HYP_HIP(head.alloc(n));
  HYP_HIP(rid.alloc(n));
  HYP_HIP(flag.alloc(4));
  const unsigned blocks = (unsigned)((n + 255) / 256);
  HYP_LAUNCH("k_jw_expand", k_jw_expand, dim3(blocks), dim3(256), 0, st, M, h, g, e_core, n1, n2, key.p, idx.p,
             re.p, im.p);
  // stable radix sort of (key, slot) over the 64 key bits
  size_t tmp_bytes = 0, tb2 = 0;
  HYP_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key.p, key2.p, idx.p, idx2.p, (int)n, 0, 64, st));
  HYP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, head.p, rid.p, (int)n, st));
  DevBuf<unsigned char> tmp;
  HYP_HIP(tmp.alloc(std::max(tmp_bytes, tb2)));
  tmp_bytes = std::max(tmp_bytes, tb2);
  {
    ProfScope ps_("hipcub_radix_sort_pauli", st);
    HYP_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, key.p, key2.p, idx.p, idx2.p, (int)n, 0, 64, st));
  }
  HYP_LAUNCH("k_run_heads", k_run_heads, dim3(blocks), dim3(256), 0, st, key2.p, n, head.p);
  HYP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, head.p, rid.p, (int)n, st));
  // number of runs = rid[n-1] + head[n-1]
  int last[2] = {0, 0};
  HYP_HIP(hipMemcpyAsync(&last[0], rid.p + (n - 1), sizeof(int), hipMemcpyDeviceToHost, st));
  HYP_HIP(hipMemcpyAsync(&last[1], head.p + (n - 1), sizeof(int), hipMemcpyDeviceToHost, st));
  HYP_HIP(hipStreamSynchronize(st));
  const int64_t nrun = (int64_t)last[0] + last[1];
  HYP_HIP(rkey.alloc(nrun));
  HYP_HIP(rc.alloc(nrun));
  HYP_HIP(keep.alloc(nrun + 1));
  HYP_HIP(pos.alloc(nrun + 1));
  HYP_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  HYP_LAUNCH("k_run_sums", k_run_sums, dim3(blocks), dim3(256), 0, st, key2.p, idx2.p, re.p, im.p, head.p, rid.p, n,
             rkey.p, rc.p, keep.p, flag.p);
  size_t tb3 = 0;
  HYP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb3, keep.p, pos.p, (int)(nrun + 1), st));
  if (tb3 > tmp_bytes) {
    HYP_HIP(hipStreamSynchronize(st));
    (void)hipFree(tmp.p);
    tmp.p = nullptr;
    HYP_HIP(tmp.alloc(tb3));
    tmp_bytes = tb3;
  }
  // keep[nrun] = 0 so pos[nrun] is the number of kept terms
  HYP_HIP(hipMemsetAsync(keep.p + nrun, 0, sizeof(int), st));
  HYP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, keep.p, pos.p, (int)(nrun + 1), st));
  int nkeep = 0, nonreal = 0;
  HYP_HIP(hipMemcpyAsync(&nkeep, pos.p + nrun, sizeof(int), hipMemcpyDeviceToHost, st));
  HYP_HIP(hipMemcpyAsync(&nonreal, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HYP_HIP(hipStreamSynchronize(st));
  if (nonreal) return fail(HYP_ERR_NONREAL, "hyp_assemble_pauli: imaginary Pauli coefficient (integrals not real-symmetric)");
  *n_out = nkeep;
  if (cap > 0 && xo && zo && co && nrun > 0) {
    HYP_LAUNCH("k_emit", k_emit, dim3((unsigned)((nrun + 255) / 256)), dim3(256), 0, st, rkey.p, rc.p, keep.p, pos.p,
               nrun, xo, zo, co, cap);
    HYP_HIP(hipGetLastError());
  }
  // the scratch is freed on return: finish the work that reads it
  HYP_HIP(hipStreamSynchronize(st));
  if (cap > 0 && nkeep > cap) return fail(HYP_ERR_ARG, "hyp_assemble_pauli: output capacity below the term count");
  return HYP_OK;
}

}  // namespace hyp

using namespace hyp;

extern "C" {

hyp_status hyp_assemble_pauli(int n_orb, const double* h_dev, const double* g_dev, double e_core,
                              uint32_t* x_dev, uint32_t* z_dev, double* c_dev, int64_t cap, int64_t* n_terms,
                              void* stream) {
  if (n_orb < 1 || n_orb > kMaxOrb) return fail(HYP_ERR_ARG, "hyp_assemble_pauli: n_orb must be in [1, 16]");
  if (!h_dev || !g_dev || !n_terms) return fail(HYP_ERR_ARG, "hyp_assemble_pauli: NULL argument");
  if (cap < 0 || (cap > 0 && (!x_dev || !z_dev || !c_dev)))
    return fail(HYP_ERR_ARG, "hyp_assemble_pauli: bad output buffers");
  return assemble_pauli(n_orb, h_dev, g_dev, e_core, x_dev, z_dev, c_dev, cap, n_terms, (hipStream_t)stream);
}

hyp_status hyp_build_hamiltonian_integrals(hyp_sector s, int n_orb, const double* h_dev, const double* g_dev,
                                           double e_core, void* stream, hyp_ham* out) {
  if (!s || !h_dev || !g_dev || !out) return fail(HYP_ERR_ARG, "hyp_build_hamiltonian_integrals: NULL argument");
  if (!sector_of(s) || sector_of(s)->M != n_orb)
    return fail(HYP_ERR_ARG, "hyp_build_hamiltonian_integrals: n_orb differs from the sector's orbital count");
  hipStream_t st = (hipStream_t)stream;
  // at most one term per expansion slot
  const int64_t cap = (int64_t)2 * n_orb * n_orb * 4 + (int64_t)n_orb * n_orb * n_orb * n_orb * 64 + 1;
  DevBuf<uint32_t> x, z;
  DevBuf<double> c;
  HYP_HIP(x.alloc(cap));
  HYP_HIP(z.alloc(cap));
  HYP_HIP(c.alloc(cap));
  int64_t n = 0;
  hyp_status r = assemble_pauli(n_orb, h_dev, g_dev, e_core, x.p, z.p, c.p, cap, &n, st);
  if (r != HYP_OK) return r;
  // the grouped table is folded and uploaded by the common build
  std::vector<uint32_t> hx, hz;
  std::vector<double> hc;
  try {
    hx.resize(n);
    hz.resize(n);
    hc.resize(n);
  } catch (...) {
    return fail(HYP_ERR_NOMEM, "hyp_build_hamiltonian_integrals: host allocation");
  }
  if (n > 0) {
    HYP_HIP(hipMemcpyAsync(hx.data(), x.p, n * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HYP_HIP(hipMemcpyAsync(hz.data(), z.p, n * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HYP_HIP(hipMemcpyAsync(hc.data(), c.p, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HYP_HIP(hipStreamSynchronize(st));
  }
  return hyp_build_hamiltonian(s, hx.data(), hz.data(), hc.data(), n, stream, out);
}

}  // extern "C"
