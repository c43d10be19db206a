// Materialised sector Hamiltonian in CSR form and its SpMV: the paper's own
// storage ("Sparse State-Vector Emulation": the Hamiltonian restricted to the
// configuration space is assembled and stored in compressed sparse row
// format, Table 1 lists its size), kept as a comparison for the matrix-free
// product.  One MI355X holds it up to about 26 qubits of the dense-integral
// workloads here (24 qubits: 1.55e9 nonzeros, 18.6 GB); at 28 qubits it
// would take 478 GB.
//
// Every row of a sector has the same number of entries,
//   L = 1 + (s_a + d_a) + (s_b + d_b) + s_a s_b
// (diagonal, alpha singles and doubles, beta singles and doubles, alpha-beta
// doubles; s = N (M - N), d = C(N,2) C(M-N,2)), each column exactly once,
// in that order.  Values come from the same folded tables as the matrix-free
// kernels: the same-spin string matrices (which hold the same-spin part of a
// diagonal, single or double), plus the other spin's number dressing of the
// singles, the alpha-beta diagonal and the alpha-beta doubles.
//
// Build: one wave per row, lanes over the row's entries (coalesced stores).
// SpMV: one wave per row, lanes over its entries, FP64 accumulation.
#include "hyp_internal.h"

#include <algorithm>
#include <new>

namespace hyp {

namespace {

__device__ inline int cpair(int p, int q) { return q * (q - 1) / 2 + p; }  // p < q

// t-th single excitation of string s (occupied index t / nemp, empty index
// t % nemp, both in ascending orbital order)
__device__ inline void nth_single(uint32_t s, uint32_t mask, int nemp, int t, int* i, int* e) {
  uint32_t occ = s, emp = ~s & mask;
  for (int j = t / nemp; j > 0; --j) occ &= occ - 1;
  for (int j = t % nemp; j > 0; --j) emp &= emp - 1;
  *i = __ffs(occ) - 1;
  *e = __ffs(emp) - 1;
}

__device__ inline int rnk(const RankTables* R, uint32_t s) { return R->lo[s & 255u] + R->hi[(s >> 8) & 255u]; }

struct CsrArgs {
  int M, na, nb, da, db;
  const uint32_t* astr;
  const uint32_t* bstr;
  const RankTables* arank;
  const RankTables* brank;
  const int* a_rank;
  const double* a_coef;
  int a_nent;
  const int* b_rank;
  const double* b_coef;
  int b_nent;
  int64_t L;
  int64_t dim;
  int* col;
  double* val;
  HamDev H;
};

__global__ void __launch_bounds__(256) k_csr_build(CsrArgs a) {
  const int64_t d = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (d >= a.dim) return;
  const int lane = threadIdx.x & 63;
  const int M = a.M;
  const uint32_t mask = (1u << M) - 1u;
  const int b = (int)(d / a.da), ac = (int)(d % a.da);
  const uint32_t bs = a.bstr[b], as = a.astr[ac];
  const HamDev& H = a.H;
  const int nemp_a = M - a.na, nemp_b = M - a.nb;
  const int sa = a.na * nemp_a, sb = a.nb * nemp_b;
  const int64_t base = d * a.L;
  const int e_alist = 1, e_blist = a.a_nent, e_ab = a.a_nent + a.b_nent - 1;
  for (int64_t e = lane; e < a.L; e += 64) {
    int c;
    double v;
    if (e == 0) {
      // diagonal: both same-spin diagonals (the beta one holds the constant)
      // and the alpha-beta diagonal sum over occupied (alpha k, beta l)
      v = a.a_coef[(int64_t)ac * a.a_nent] + a.b_coef[(int64_t)b * a.b_nent];
      uint32_t ok = as;
      while (ok) {
        const int k = __ffs(ok) - 1;
        ok &= ok - 1;
        uint32_t ol = bs;
        while (ol) {
          const int l = __ffs(ol) - 1;
          ol &= ol - 1;
          v += H.dC[k * 32 + (l + M)];
        }
      }
      c = (int)d;
    } else if (e < e_blist) {
      // alpha list entry: single or double of the alpha string, same beta row
      const int x = (int)(e - e_alist) + 1;
      c = b * a.da + a.a_rank[(int64_t)ac * a.a_nent + x];
      v = a.a_coef[(int64_t)ac * a.a_nent + x];
      if (x - 1 < sa) {
        // single: the beta-occupation dressing, sign (-1)^{popc(sJ & alpha)}
        int i, em;
        nth_single(as, mask, nemp_a, x - 1, &i, &em);
        const int pid = cpair(min(i, em), max(i, em)), O = (i == max(i, em)) ? 1 : 0;
        const double* B = H.sB + (size_t)(pid * 2 + O) * 32;
        double w = 0.0;
        uint32_t ol = bs;
        while (ol) {
          const int l = __ffs(ol) - 1;
          ol &= ol - 1;
          w += B[l + M];
        }
        v += (__popc(H.sJ[pid] & as) & 1) ? -w : w;
      }
    } else if (e < e_ab) {
      // beta list entry: single or double of the beta string, same alpha column
      const int x = (int)(e - e_blist) + 1;
      c = a.b_rank[(int64_t)b * a.b_nent + x] * a.da + ac;
      v = a.b_coef[(int64_t)b * a.b_nent + x];
      if (x - 1 < sb) {
        // single: the alpha-occupation dressing
        int i, em;
        nth_single(bs, mask, nemp_b, x - 1, &i, &em);
        const int pb = cpair(min(i, em), max(i, em)), Ob = (i == max(i, em)) ? 1 : 0;
        const double* B = H.sB + (size_t)((kMaxPairs + pb) * 2 + Ob) * 32;
        double w = 0.0;
        uint32_t ok = as;
        while (ok) {
          const int k = __ffs(ok) - 1;
          ok &= ok - 1;
          w += B[k];
        }
        v += (__popc((H.sJ[kMaxPairs + pb] >> M) & bs) & 1) ? -w : w;
      }
    } else {
      // alpha-beta double: beta single jb times alpha single x
      const int t = (int)(e - e_ab);
      const int jb = t / sa, x = t % sa;
      int ib, eb, ia, ea;
      nth_single(bs, mask, nemp_b, jb, &ib, &eb);
      nth_single(as, mask, nemp_a, x, &ia, &ea);
      const int pb = cpair(min(ib, eb), max(ib, eb)), Ob = (ib == max(ib, eb)) ? 1 : 0;
      const int pa = cpair(min(ia, ea), max(ia, ea)), Oa = (ia == max(ia, ea)) ? 1 : 0;
      const uint32_t sg = (__popc((H.abJb[pb] >> M) & bs) ^ __popc(H.abJa[pa] & as)) & 1u;
      const double f = H.abF[((size_t)pa * kMaxPairs + pb) * 4 + Oa * 2 + Ob];
      v = sg ? -f : f;
      const uint32_t b2 = bs ^ (1u << ib) ^ (1u << eb), a2 = as ^ (1u << ia) ^ (1u << ea);
      c = rnk(a.brank, b2) * a.da + rnk(a.arank, a2);
    }
    a.col[base + e] = c;
    a.val[base + e] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_csr_spmv(const int64_t* __restrict__ rp, const int* __restrict__ col,
                                                  const double* __restrict__ val, const T* __restrict__ x,
                                                  T* __restrict__ y, int64_t nrow) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nrow) return;
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  const int64_t e1 = rp[r + 1];
  for (int64_t e = rp[r] + lane; e < e1; e += 64) {
    if (sizeof(T) == 4)
      acc += (double)((float)val[e] * (float)x[col[e]]);
    else
      acc += val[e] * (double)x[col[e]];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) y[r] = (T)acc;
}

__global__ void k_csr_rowptr(int64_t* rp, int64_t n, int64_t L) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
    rp[i] = i * L;
}

}  // namespace
}  // namespace hyp

using namespace hyp;

struct hyp_csr_s {
  int64_t dim = 0, nnz = 0;
  int64_t* rp = nullptr;
  int* col = nullptr;
  double* val = nullptr;
};

extern "C" {

hyp_status hyp_csr_destroy(hyp_csr m) {
  if (!m) return HYP_OK;
  (void)hipFree(m->rp);
  (void)hipFree(m->col);
  (void)hipFree(m->val);
  delete m;
  return HYP_OK;
}

int64_t hyp_csr_nnz(hyp_csr m) { return m ? m->nnz : -1; }

hyp_status hyp_csr_build(hyp_ham hh, void* stream, hyp_csr* out) {
  if (!hh || !out) return fail(HYP_ERR_ARG, "hyp_csr_build: NULL argument");
  Ham* Hm = ham_of(hh);
  if (!Hm->structured)
    return fail(HYP_ERR_UNSUPPORTED, "hyp_csr_build: only two-body number-conserving Hamiltonians are materialised");
  HamWork* W = work_of(hh);
  Sector* S = Hm->sec;
  const int sa = S->na * (S->M - S->na), sb = S->nb * (S->M - S->nb);
  const int64_t L = 1 + (int64_t)(W->a_nent - 1) + (W->b_nent - 1) + (int64_t)sa * sb;
  const int64_t nnz = S->dim * L;
  const size_t bytes = (size_t)nnz * (sizeof(int) + sizeof(double)) + (size_t)(S->dim + 1) * sizeof(int64_t);
  size_t free_b = 0, total_b = 0;
  HYP_HIP(hipMemGetInfo(&free_b, &total_b));
  if (bytes + ((size_t)2 << 30) > free_b)
    return fail(HYP_ERR_NOMEM, "hyp_csr_build: the CSR needs " + std::to_string(bytes) + " bytes, " +
                                   std::to_string(free_b) + " free on the device");
  hipStream_t st = (hipStream_t)stream;
  hyp_csr m = new (std::nothrow) hyp_csr_s;
  if (!m) return fail(HYP_ERR_NOMEM, "hyp_csr_build: host allocation");
  m->dim = S->dim;
  m->nnz = nnz;
  hipError_t e = hipMalloc(&m->rp, (S->dim + 1) * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&m->col, (size_t)nnz * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&m->val, (size_t)nnz * sizeof(double));
  if (e != hipSuccess) {
    hyp_csr_destroy(m);
    return hip_fail(e, "hyp_csr_build: allocation");
  }
  HYP_LAUNCH("k_csr_rowptr", k_csr_rowptr, dim3(1024), dim3(256), 0, st, m->rp, S->dim, L);
  CsrArgs a;
  a.M = S->M;
  a.na = S->na;
  a.nb = S->nb;
  a.da = (int)S->da;
  a.db = (int)S->db;
  a.astr = S->d_astr;
  a.bstr = S->d_bstr;
  a.arank = S->d_arank;
  a.brank = S->d_brank;
  a.a_rank = W->a_rank;
  a.a_coef = W->a_coef;
  a.a_nent = W->a_nent;
  a.b_rank = W->b_rank;
  a.b_coef = W->b_coef;
  a.b_nent = W->b_nent;
  a.L = L;
  a.dim = S->dim;
  a.col = m->col;
  a.val = m->val;
  a.H = Hm->dev;
  HYP_LAUNCH("k_csr_build", k_csr_build, dim3((unsigned)((S->dim + 3) / 4)), dim3(256), 0, st, a);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    hyp_csr_destroy(m);
    return hip_fail(e, "hyp_csr_build: build kernel");
  }
  *out = m;
  return HYP_OK;
}

hyp_status hyp_csr_apply(hyp_csr m, hyp_dtype dtype, const void* psi, void* sigma, void* stream) {
  if (!m || !psi || !sigma) return fail(HYP_ERR_ARG, "hyp_csr_apply: NULL argument");
  if (psi == sigma) return fail(HYP_ERR_ARG, "hyp_csr_apply: psi and sigma alias");
  hipStream_t st = (hipStream_t)stream;
  const dim3 g((unsigned)((m->dim + 3) / 4));
  if (dtype == HYP_F64)
    HYP_LAUNCH("k_csr_spmv", k_csr_spmv<double>, g, dim3(256), 0, st, m->rp, m->col, m->val, (const double*)psi,
               (double*)sigma, m->dim);
  else if (dtype == HYP_F32)
    HYP_LAUNCH("k_csr_spmv", k_csr_spmv<float>, g, dim3(256), 0, st, m->rp, m->col, m->val, (const float*)psi,
               (float*)sigma, m->dim);
  else
    return fail(HYP_ERR_ARG, "hyp_csr_apply: bad dtype");
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

hyp_status hyp_csr_export(hyp_csr m, int64_t* row_ptr, int32_t* col, double* val) {
  if (!m || !row_ptr || !col || !val) return fail(HYP_ERR_ARG, "hyp_csr_export: NULL argument");
  HYP_HIP(hipDeviceSynchronize());
  HYP_HIP(hipMemcpy(row_ptr, m->rp, (m->dim + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  HYP_HIP(hipMemcpy(col, m->col, (size_t)m->nnz * sizeof(int), hipMemcpyDeviceToHost));
  HYP_HIP(hipMemcpy(val, m->val, (size_t)m->nnz * sizeof(double), hipMemcpyDeviceToHost));
  return HYP_OK;
}

}  // extern "C"
