// Matrix-free sigma = P_S H P_S psi on gfx950 for a Pauli-sum Hamiltonian
// grouped by X-mask (paper, "Sparse State-Vector Emulation": the sparse
// Hamiltonian-state product that dominates ADAPT-VQE; here the CSR matrix is
// never formed, each output amplitude pulls from its connected inputs).
//
// Build: the Pauli terms are grouped by x.  For an in-sector output d, a term
// contributes c' (-1)^{popc(z & d)} psi[d xor x], c' = c (-1)^{n_Y/2}.  For a
// two-body number-conserving Hamiltonian every group folds, exactly, into a
// small closed form over d's occupations (HamDev in hyp_internal.h).  The
// per-output work is then split by which spin the excitation touches:
//   same-spin part  (diagonal in the other spin's string):  a sparse
//       string-space matrix applied to whole rows -- kernel k_same_spin, run
//       once on psi (beta rows) and once on psi^T (alpha rows);
//   mixed part (alpha-beta doubles, the other-spin number dressing of singles,
//       the alpha-beta diagonal): kernel k_mixed, one workgroup per beta row
//       with the needed source rows staged through LDS.
// Any real Pauli sum outside that class falls back to k_generic, a
// term-by-term pull over X-groups.
#include "hyp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <type_traits>

namespace hyp {

// ---------------------------------------------------------------- helpers

__host__ __device__ inline int pair_id(int p, int q) { return q * (q - 1) / 2 + p; }  // p < q

__host__ __device__ inline int choose_small(int m, int k) {
  // C(m, k) for m < 16, k <= 4 (quad ids)
  if (k > m || m < 0) return 0;
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (m - k + i) / i;
  return r;
}

__host__ __device__ inline int quad_id(int o0, int o1, int o2, int o3) {
  return choose_small(o0, 1) + choose_small(o1, 2) + choose_small(o2, 3) + choose_small(o3, 4);
}

template <typename T>
struct Acc;  // storage type -> product rules
template <>
struct Acc<double> {
  __device__ static inline double prod(double c, double v) { return c * v; }
  __device__ static inline double load(const double* p) { return *p; }
};
template <>
struct Acc<float> {
  // FP32 product, FP64 accumulation by the caller
  __device__ static inline double prod(double c, float v) { return (double)((float)c * v); }
  __device__ static inline double prod(float c, float v) { return (double)(c * v); }
  __device__ static inline double load(const float* p) { return (double)*p; }
};

__device__ inline double flip(double v, uint32_t odd) {
  // multiply by (-1)^odd without a multiply: toggle the sign bit
  uint64_t u = __double_as_longlong(v) ^ ((uint64_t)(odd & 1u) << 63);
  return __longlong_as_double(u);
}

// ---------------------------------------------------------------- transpose

// in[rows][cols] -> out[cols][rows], 64x64 tiles through LDS.  With row_nz
// and col_nz (cleared beforehand) it also records the support of `in` at
// row and column granularity: a wave that sees a nonzero amplitude of a row
// (input phase) or of a column (output phase) sets that row's or column's
// flag to 1.
template <typename T>
__global__ void k_transpose(const T* __restrict__ in, T* __restrict__ out, int rows, int cols,
                            uint32_t* __restrict__ row_nz, uint32_t* __restrict__ col_nz) {
  __shared__ T tile[64][65];
  int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 256 threads: 4 rows per pass
  for (int r = ty; r < 64; r += 4) {
    int rr = r0 + r, cc = c0 + tx;
    T v = T(0);
    if (rr < rows && cc < cols) tile[r][tx] = v = in[(int64_t)rr * cols + cc];
    if (row_nz && __ballot(v != T(0)) && tx == 0) row_nz[rr] = 1u;
  }
  __syncthreads();
  for (int c = ty; c < 64; c += 4) {
    int cc = c0 + c, rr = r0 + tx;
    T v = T(0);
    if (rr < rows && cc < cols) out[(int64_t)cc * rows + rr] = v = tile[tx][c];
    if (col_nz && __ballot(v != T(0)) && tx == 0) col_nz[cc] = 1u;
  }
}

__global__ void k_clear_u32(uint32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Support-restricted copy of a same-spin matrix: row r keeps, in order, the
// entries whose source row has a nonzero flag; c_n[r] = their count.  One
// wave per row.
__global__ void __launch_bounds__(256) k_ss_compact(const int* __restrict__ rank, const double* __restrict__ coef,
                                                    int nent, int nuse, int nrow, const uint32_t* __restrict__ src_nz,
                                                    int* __restrict__ c_rank, double* __restrict__ c_coef,
                                                    int* __restrict__ c_n) {
  // rows of nent entries (the stride), of which the first nuse are compacted
  const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (row >= nrow) return;
  const int lane = threadIdx.x & 63;
  const int64_t base = (int64_t)row * nent;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int n = 0;
  for (int e0 = 0; e0 < nuse; e0 += 64) {
    const int e = e0 + lane;
    int r = 0;
    bool keep = false;
    if (e < nuse) {
      r = rank[base + e];
      keep = src_nz[r] != 0u;
    }
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int64_t pos = base + n + __popcll(m & below);
      c_rank[pos] = r;
      c_coef[pos] = coef[base + e];
    }
    n += __popcll(m);
  }
  if (lane == 0) c_n[row] = n;
}

// ---------------------------------------------------------------- same-spin rows

struct SameSpinArgs {
  int* list_rank;         // [nrow][nent] source row of each entry
  double* list_coef;      // [nrow][nent] coefficient of each entry
  int nent;
  int nrow;
  int M, nel;             // orbitals, electrons of the row spin
  int spin;               // 0 alpha rows, 1 beta rows
  const uint32_t* rstr;   // [nrow] row strings
  const RankTables* rrank;
  double constant;        // added to every diagonal (the identity term), once
  HamDev H;
};

constexpr int kSameSpinMax = 1 + 64 + 784;  // self + singles + doubles for M <= 16
constexpr int kSSThreads = 256;

// Row r of Hs, the same-spin part of H as a sparse matrix over strings of
// one spin (pure-spin diagonal, singles with same-spin number dressing,
// same-spin doubles), evaluated from the folded X-group tables and stored
// as (source row, coefficient) entries.  Built once per Hamiltonian: one
// workgroup per row string.
__global__ void __launch_bounds__(kSSThreads) k_ss_build(SameSpinArgs a) {
  __shared__ int s_rank[kSameSpinMax];
  __shared__ double s_coef[kSameSpinMax];
  __shared__ int s_n;
  const int row = blockIdx.x;
  const uint32_t s = a.rstr[row];
  const int off = a.spin * a.M;  // qubit offset of this spin
  const uint32_t smask = (1u << a.M) - 1u;
  if (threadIdx.x == 0) {
    // self term
    double e = a.constant;
    uint32_t o1 = s;
    while (o1) {
      int k = __ffs(o1) - 1;
      o1 &= o1 - 1;
      e += a.H.dB[k + off];
      uint32_t o2 = o1;
      while (o2) {
        int l = __ffs(o2) - 1;
        o2 &= o2 - 1;
        e += a.H.dC[(k + off) * 32 + (l + off)];
      }
    }
    s_rank[0] = row;
    s_coef[0] = e;
    s_n = 1;
  }
  __syncthreads();
  // singles: thread t handles pair (i occupied, a empty) number t
  {
    const int nemp = a.M - a.nel;
    const int ns = a.nel * nemp;
    for (int t = threadIdx.x; t < ns; t += blockDim.x) {
      int io = t / nemp, ie = t % nemp;
      // io-th occupied and ie-th empty orbital
      uint32_t occ = s, emp = ~s & smask;
      for (int j = 0; j < io; ++j) occ &= occ - 1;
      for (int j = 0; j < ie; ++j) emp &= emp - 1;
      int i = __ffs(occ) - 1, e = __ffs(emp) - 1;
      int p = min(i, e), q = max(i, e);
      int pid = pair_id(p, q);
      int O = (i == q) ? 1 : 0;
      const int base = (a.spin * kMaxPairs + pid);
      double v = a.H.sA[base * 2 + O];
      const double* B = a.H.sB + (size_t)(base * 2 + O) * 32;
      uint32_t oc = s;
      while (oc) {
        int k = __ffs(oc) - 1;
        oc &= oc - 1;
        v += B[k + off];
      }
      uint32_t J = a.H.sJ[base] >> off;
      v = flip(v, __popc(J & s));
      uint32_t t2 = s ^ (1u << i) ^ (1u << e);
      s_rank[1 + t] = a.rrank->lo[t2 & 255u] + a.rrank->hi[(t2 >> 8) & 255u];
      s_coef[1 + t] = v;
    }
    // doubles: (i<j occupied) x (a<b empty)
    const int no2 = a.nel * (a.nel - 1) / 2, ne2 = nemp * (nemp - 1) / 2;
    const int nd = no2 * ne2;
    for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      int po = t / ne2, pe = t % ne2;
      // decode pair index po into (jo > io) among occupied list by colex
      int jo = 1;
      while ((jo + 1) * jo / 2 <= po) ++jo;
      int io = po - jo * (jo - 1) / 2;
      int je = 1;
      while ((je + 1) * je / 2 <= pe) ++je;
      int ie = pe - je * (je - 1) / 2;
      uint32_t occ = s, emp = ~s & smask;
      int oi = -1, oj = -1, ea = -1, eb = -1;
      for (int c = 0; occ; ++c) {
        int k = __ffs(occ) - 1;
        occ &= occ - 1;
        if (c == io) oi = k;
        if (c == jo) oj = k;
      }
      for (int c = 0; emp; ++c) {
        int k = __ffs(emp) - 1;
        emp &= emp - 1;
        if (c == ie) ea = k;
        if (c == je) eb = k;
      }
      // sorted quad and occupied pattern
      int q4[4] = {oi, oj, ea, eb};
      for (int x = 1; x < 4; ++x)
        for (int y = x; y > 0 && q4[y - 1] > q4[y]; --y) {
          int tmp = q4[y];
          q4[y] = q4[y - 1];
          q4[y - 1] = tmp;
        }
      int O4 = 0;
      for (int x = 0; x < 4; ++x)
        if (q4[x] == oi || q4[x] == oj) O4 |= 1 << x;
      int qid = quad_id(q4[0], q4[1], q4[2], q4[3]);
      const int base = a.spin * kMaxQuads + qid;
      double v = a.H.wF[(size_t)base * 16 + O4];
      uint32_t J = a.H.wJ[base] >> off;
      v = flip(v, __popc(J & s));
      uint32_t t2 = s ^ (1u << oi) ^ (1u << oj) ^ (1u << ea) ^ (1u << eb);
      s_rank[1 + ns + t] = a.rrank->lo[t2 & 255u] + a.rrank->hi[(t2 >> 8) & 255u];
      s_coef[1 + ns + t] = v;
    }
    if (threadIdx.x == 0) s_n = 1 + ns + nd;
  }
  __syncthreads();
  const int n = s_n;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    a.list_rank[(int64_t)row * a.nent + e] = s_rank[e];
    a.list_coef[(int64_t)row * a.nent + e] = s_coef[e];
  }
}

struct SSApplyArgs {
  const void* in;           // [nrow][ncol] storage T
  double* out;              // [nrow][ncol] FP64 partial
  const int* list_rank;
  const double* list_coef;
  const int* list_n;        // per-row entry counts (support-restricted lists), or null: nuse each
  int nent, nrow, ncol;     // nent: the lists' row stride
  int nuse;                 // entries used per row (all nent, or the singles and diagonal head)
  int ntiles, nrb;          // 64-column tiles, 4-row blocks
  // columns [c0, c0 + nc) (a band; 0, ncol for all) and, for the core path,
  // the band's per-core products: row r adds Y[yoff[r][m] * ldy + c - c0]
  // over its npair cores m (skipped where cnz flags a core as zero)
  int c0, nc;
  const double* Y;
  int64_t ldy;
  const int* yoff;
  int npair, S;
  const int* cnz;
  const int* row_any;       // support skipping: 0 where the row has nothing (written as zeros)
  const int* sel;           // support skipping: run only where *sel == 1 (the core path is selected)
};

// out[r][c] = sum_e coef[r][e] in[rank[r][e]][c].  Each wave owns one output
// row and 64 consecutive columns, so its entry list is wave-uniform.  The
// workgroup -> (tile, rows) map is XCD-aware: workgroups are dispatched to
// the 8 XCDs round-robin, so block b runs on XCD b % 8; consecutive blocks
// of one XCD take consecutive row blocks of the same 64-column tile, and the
// tile's slab of the input (nrow x 64 amplitudes) stays in that XCD's L2.
template <typename T, bool kY>
__global__ void __launch_bounds__(256) k_ss_apply(SSApplyArgs a) {
  const int b = blockIdx.x;
  const int xcd = b & 7, j = b >> 3;
  const int tile = (j / a.nrb) * 8 + xcd;
  const int rb = j % a.nrb;
  if (tile >= a.ntiles) return;
  const int row = rb * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= a.nrow) return;
  const int col = a.c0 + tile * 64 + (threadIdx.x & 63);
  const bool live = col < a.c0 + a.nc && col < a.ncol;
  const int colc = live ? col : a.c0;
  const int* __restrict__ rk = a.list_rank + (int64_t)row * a.nent;
  const double* __restrict__ cf = a.list_coef + (int64_t)row * a.nent;
  const T* __restrict__ in = (const T*)a.in;
  if (kY && a.sel && *a.sel != 1) return;
  if (kY && a.row_any && __builtin_amdgcn_readfirstlane(a.row_any[row]) == 0) {
    if (live) a.out[(int64_t)row * a.ncol + col] = 0.0;
    return;
  }
  const int nent = a.list_n ? __builtin_amdgcn_readfirstlane(a.list_n[row]) : a.nuse;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int e = 0;
  // eight independent loads in flight per wave
  for (; e + 8 <= nent; e += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int r = __builtin_amdgcn_readfirstlane(rk[e + u]);
      v[u] = in[(int64_t)r * a.ncol + colc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u & 3] += Acc<T>::prod(cf[e + u], v[u]);
  }
  for (; e < nent; ++e) {
    const int r = __builtin_amdgcn_readfirstlane(rk[e]);
    acc[0] += Acc<T>::prod(cf[e], in[(int64_t)r * a.ncol + colc]);
  }
  double sum = (acc[0] + acc[2]) + (acc[1] + acc[3]);
  if constexpr (kY) {
    // the row's same-spin doubles: its npair cores' product rows, in order
    const int* __restrict__ yo = a.yoff + (int64_t)row * a.npair;
    const int64_t cy = colc - a.c0;
    int m = 0;
    for (; m + 8 <= a.npair; m += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int o = __builtin_amdgcn_readfirstlane(yo[m + u]);
        const bool z = a.cnz && a.cnz[o / a.S] == 0;
        v[u] = z ? 0.0 : __builtin_nontemporal_load(&a.Y[(int64_t)o * a.ldy + cy]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; m < a.npair; ++m) {
      const int o = __builtin_amdgcn_readfirstlane(yo[m]);
      if (!(a.cnz && a.cnz[o / a.S] == 0)) sum += __builtin_nontemporal_load(&a.Y[(int64_t)o * a.ldy + cy]);
    }
  }
  if (live) a.out[(int64_t)row * a.ncol + col] = sum;
}

// ---------------------------------------------------------------- same-spin doubles through cores
//
// Every same-spin double pairs two strings that share exactly one core: the
// (N - 2)-electron string K = I & J, the two strings being K plus two
// disjoint pairs of the F = M - N + 2 orbitals outside K (the core's S =
// C(F, 2) slots; tables of core_gram.hip).  So the doubles part of the
// same-spin product, sum over r' of H[r][r'] in[r'][c], is for each core a
// small dense product
//   Y_K[i][c] = sum_j W_K[i][j] in[K + slot j][c],
// W_K[i][j] the coefficient of the double from K + slot j into K + slot i
// (zero unless the slots are disjoint), and row r = K + slot i gathers
// Y_K[i] over its C(N, 2) cores (k_ss_apply with kY).  A row's 784 gathered
// sources (16 orbitals, 8 electrons) become 28 rows of Y, and each source
// row is read once per core that holds it.
//
// k_ss_core: one 256-thread workgroup per core and column band.  W_K (S <=
// 48, padded to 48) is evaluated from the folded double tables into
// registers as FP64 MFMA A operands (lane l: row 16 b + (l & 15), column 4 s
// + (l >> 4)); the band's 64-column chunks of the core's S source rows are
// copied into two alternating LDS buffers (direct copies, the next chunk in
// flight) and wave w forms the 48 x 16 block of Y for chunk columns
// 16 w .. 16 w + 15 with v_mfma_f64_16x16x4_f64 (element e of lane l holds
// row 16 b + (l >> 4) + 4 e, column l & 15).
struct SSCoreArgs {
  const double* in;        // [nrow][ld] FP64 rows (psi, or psi^T for the alpha rows)
  int64_t ld;
  int dma;                 // 1: in 16-byte aligned, ld and c0 even (direct copies)
  const int* rows;         // [ncore][S] source row of each slot
  const uint32_t* masks;   // [ncore] the core's orbitals
  int ncore, S, M, spin;
  int64_t per_xcd;         // ceil(ncore / 8): consecutive cores on one XCD
  const uint32_t* wJ;      // folded same-spin double tables (HamDev)
  const double* wF;
  int c0, nc;              // the band's columns
  double* Y;               // [ncore][S][ldy]
  int64_t ldy;
  const int* cnz;          // support skipping: [ncore] 0 for a core with no row in the support (null: every core)
  const int* sel;          // support skipping: run only where *sel == 1
};

// Support skipping, per spin and product: the core path where at least a
// quarter of the source rows are in psi's support, else the grouped lists
// (which then compact to few sources per group while every core still forms
// its whole band).  One workgroup: *sel = (4 * flagged rows >= nrow).
__global__ void __launch_bounds__(1024) k_ss_select(const uint32_t* __restrict__ flags, int nrow,
                                                    int* __restrict__ sel) {
  __shared__ int s_n[16];
  int n = 0;
  for (int r = threadIdx.x; r < nrow; r += blockDim.x) n += flags[r] != 0u ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) n += __shfl_down(n, o, 64);
  if ((threadIdx.x & 63) == 0) s_n[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_n[w];
    *sel = 4 * t >= nrow ? 1 : 0;
  }
}

// Support skipping, once per spin and product: cnz[core] = 1 if some source
// row of the core is in psi's support (one thread per core) ...
__global__ void __launch_bounds__(256) k_core_flags(const int* __restrict__ rows, int ncore, int S,
                                                    const uint32_t* __restrict__ rflag, int* __restrict__ cnz) {
  const int core = blockIdx.x * blockDim.x + threadIdx.x;
  if (core >= ncore) return;
  int any = 0;
  for (int j = 0; j < S && !any; ++j) any = rflag[rows[(int64_t)core * S + j]] != 0u;
  cnz[core] = any;
}

// ... and row_any[r] = 1 if row r keeps a single or diagonal entry or one
// of its cores is flagged (one thread per row).
__global__ void __launch_bounds__(256) k_row_any(const int* __restrict__ yoff, int npair, int S,
                                                 const int* __restrict__ cnz, const int* __restrict__ list_n,
                                                 int nrow, int* __restrict__ row_any) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrow) return;
  int any = list_n[row] > 0;
  for (int m = 0; m < npair && !any; ++m) any = cnz[yoff[(int64_t)row * npair + m] / S] != 0;
  row_any[row] = any;
}
constexpr int kCoreC = 64;                          // columns per staged chunk
constexpr int kCoreLd = kCoreC + 2;                 // LDS row stride in doubles
constexpr int kCorePieces = 48 * (kCoreLd / 2);     // 16-byte pieces per buffer
constexpr uint32_t kCoreBuf = kCorePieces * 16u;    // 25,344 bytes
constexpr int kCorePer = (kCorePieces + 255) / 256;

__global__ void __launch_bounds__(256) k_ss_core(SSCoreArgs a) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_row[48];
  __shared__ int s_comp[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t b = blockIdx.x;
  const int64_t core = (b & 7) * a.per_xcd + (b >> 3);
  if (core >= a.ncore) return;
  // support skipping: a core none of whose rows is in psi's support (flags
  // of k_core_flags) has a zero product; its gatherers skip it
  if (a.sel && *a.sel != 1) return;
  if (a.cnz && a.cnz[core] == 0) return;
  const int S = a.S;
  const uint32_t K = a.masks[core];
  if (tid < 48) s_row[tid] = tid < S ? a.rows[core * S + tid] : -1;
  if (tid == 0) {
    int nf = 0;
    for (int o = 0; o < a.M; ++o)
      if (!(K >> o & 1u)) s_comp[nf++] = o;
  }
  __syncthreads();
  // W_K as MFMA A operands
  const int mr = lane & 15, mk = lane >> 4;
  const int off = a.spin * a.M;
  auto slot_pair = [&](int i, int& p, int& q) {
    int wv = 1;
    while ((wv + 1) * wv / 2 <= i) ++wv;
    p = s_comp[i - wv * (wv - 1) / 2];
    q = s_comp[wv];
  };
  double wreg[3][12];
#pragma unroll
  for (int bi = 0; bi < 3; ++bi)
#pragma unroll
    for (int st = 0; st < 12; ++st) {
      const int i = 16 * bi + mr, j = 4 * st + mk;
      double v = 0.0;
      if (i < S && j < S) {
        int p, q, sa, sb;
        slot_pair(i, p, q);
        slot_pair(j, sa, sb);
        if (p != sa && p != sb && q != sa && q != sb) {
          int q4[4] = {p, q, sa, sb};
#pragma unroll
          for (int x = 1; x < 4; ++x)
#pragma unroll
            for (int y = x; y > 0; --y)
              if (q4[y - 1] > q4[y]) {
                const int t = q4[y];
                q4[y] = q4[y - 1];
                q4[y - 1] = t;
              }
          int O4 = 0;
#pragma unroll
          for (int x = 0; x < 4; ++x)
            if (q4[x] == p || q4[x] == q) O4 |= 1 << x;
          const int base = a.spin * kMaxQuads + quad_id(q4[0], q4[1], q4[2], q4[3]);
          const uint32_t J = a.wJ[base] >> off;
          v = flip(a.wF[(size_t)base * 16 + O4], __popc(J & (K | (1u << p) | (1u << q))));
        }
      }
      wreg[bi][st] = v;
    }
  // staging pieces: LDS piece q = j * 256 + tid holds columns 2 col, 2 col + 1
  // of slot row q / 33 (col = q % 33; col 32 pads)
  int poff[kCorePer];
#pragma unroll
  for (int j = 0; j < kCorePer; ++j) {
    const int q = j * 256 + tid;
    const int row = q / (kCoreLd / 2), col = q - row * (kCoreLd / 2);
    const bool act = q < kCorePieces && col < kCoreC / 2 && s_row[row] >= 0;
    poff[j] = act ? (int)((int64_t)s_row[row] * a.ld + 2 * col) : -1;
  }
  const uint32_t buf0 = lds_addr(smem), buf1 = buf0 + kCoreBuf;
  // columns [k0, k0 + kn) of the slot rows through registers, zeros past kn
  // and on rows without a slot
  auto stage_regs = [&](uint32_t buf, int k0, int kn) {
#pragma unroll
    for (int j = 0; j < kCorePer; ++j) {
      const int q = j * 256 + tid;
      const int row = q / (kCoreLd / 2), col = q - row * (kCoreLd / 2);
      if (q < kCorePieces && col < kCoreC / 2) {
        f64x2 v = {0.0, 0.0};
        if (s_row[row] >= 0) {
          const double* src = a.in + (int64_t)s_row[row] * a.ld + k0;
          if (2 * col < kn) v.x = src[2 * col];
          if (2 * col + 1 < kn) v.y = src[2 * col + 1];
        }
        *(__attribute__((address_space(3))) f64x2*)(uintptr_t)(buf + (uint32_t)q * 16u) = v;
      }
    }
  };
  auto issue = [&](uint32_t buf, int k0) {
#pragma unroll
    for (int j = 0; j < kCorePer; ++j) {
      const int base = j * 256 + w * 64;  // wave-uniform first piece
      if (base < kCorePieces) {
        const uint32_t dst = (uint32_t)__builtin_amdgcn_readfirstlane(buf + (uint32_t)base * 16u);
        if (poff[j] >= 0) dma16(dst, a.in + poff[j] + k0);
      }
    }
  };
  f64x4 acc[3];
  auto compute = [&](uint32_t buf) {
#pragma unroll
    for (int bi = 0; bi < 3; ++bi) acc[bi] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 12; ++st) {
      const double bv = lds_load<double>(buf + (uint32_t)((4 * st + mk) * kCoreLd + 16 * w + mr) * 8u);
#pragma unroll
      for (int bi = 0; bi < 3; ++bi) acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(wreg[bi][st], bv, acc[bi], 0, 0, 0);
    }
  };
  // Y rows of the chunk at column k0 (kn valid columns)
  auto store = [&](int k0, int kn) {
    const int cc = 16 * w + mr;
    if (cc < kn) {
#pragma unroll
      for (int bi = 0; bi < 3; ++bi)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = 16 * bi + mk + 4 * e;
          if (i < S) __builtin_nontemporal_store(acc[bi][e], &a.Y[(core * S + i) * a.ldy + (k0 - a.c0) + cc]);
        }
    }
  };
  const int nfull = a.dma ? a.nc / kCoreC : 0;
  // every piece of both buffers cleared once: rows without a slot and pad
  // columns stay zero under the direct copies (their W columns are zero)
  stage_regs(buf0, 0, 0);
  stage_regs(buf1, 0, 0);
  __syncthreads();
  if (nfull > 0) {
    issue(buf0, a.c0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  for (int ch = 0; ch < nfull; ++ch) {
    const uint32_t cur = (ch & 1) ? buf1 : buf0, nxt = (ch & 1) ? buf0 : buf1;
    if (ch + 1 < nfull) issue(nxt, a.c0 + (ch + 1) * kCoreC);
    // chunk ch - 1's rows of Y, stored here so that they and the copy are
    // in flight during this chunk's products
    if (ch > 0) store(a.c0 + (ch - 1) * kCoreC, kCoreC);
    compute(cur);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // chunk ch + 1 copied by every wave; chunk ch's reads done
  }
  if (nfull > 0) store(a.c0 + (nfull - 1) * kCoreC, kCoreC);
  for (int k0 = a.c0 + nfull * kCoreC; k0 < a.c0 + a.nc; k0 += kCoreC) {
    const int kn = min(kCoreC, a.c0 + a.nc - k0);
    stage_regs(buf0, k0, kn);
    __syncthreads();
    compute(buf0);
    store(k0, kn);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- grouped same-spin rows
//
// The same-spin product is a sparse string-space matrix times a dense
// matrix; a row's 1 + s + d sources (849 at 16 orbitals and 8 electrons)
// overlap heavily with those of the rows next to it in colex order.  Groups
// of kSSG consecutive output rows therefore share one source list, the union
// of their rows' sources (362 sources per row instead of 849 at that size),
// each source with the kSSG coefficients of the group's rows (zero where a
// row does not reach it).  One wave per (group, 64 columns) loads each union
// source once and updates kSSG accumulators: 2.3x fewer gathered loads for
// 3.4x the FMAs, which the vector ALU has to spare (FP64 storage; the FP32
// pass keeps the per-row kernel).
constexpr int kSSG = 8;            // output rows per group
constexpr int kSSGWords = 512;     // bitmap words over source rows (C(16, 8) = 12,870 < 16,384)

__device__ inline void ssg_mark(const int* __restrict__ rank, int nent, int nrow, int g, uint32_t* bm) {
  for (int i = threadIdx.x; i < kSSGWords; i += blockDim.x) bm[i] = 0u;
  __syncthreads();
  const int r0 = g * kSSG, nr = min(kSSG, nrow - r0);
  for (int i = threadIdx.x; i < nr * nent; i += blockDim.x) {
    const int src = rank[(int64_t)r0 * nent + i];
    atomicOr(&bm[src >> 5], 1u << (src & 31));
  }
  __syncthreads();
}

// cnt[g] = size of the union of group g's sources.  One workgroup per group.
__global__ void __launch_bounds__(256) k_ssg_count(const int* __restrict__ rank, int nent, int nrow,
                                                   int* __restrict__ cnt) {
  __shared__ uint32_t bm[kSSGWords];
  __shared__ int s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  ssg_mark(rank, nent, nrow, blockIdx.x, bm);
  int c = 0;
  for (int i = threadIdx.x; i < kSSGWords; i += blockDim.x) c += __popc(bm[i]);
  atomicAdd(&s_sum, c);
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = s_sum;
}

// Group g's union list from position off[g] on, in ascending source rank:
// urank[u] and the group's row coefficients ucoef[u][0..kSSG) (zero where a
// row does not reach the source).  One workgroup per group.
__global__ void __launch_bounds__(256) k_ssg_fill(const int* __restrict__ rank, const double* __restrict__ coef,
                                                  int nent, int nrow, const int64_t* __restrict__ off,
                                                  int* __restrict__ urank, double* __restrict__ ucoef) {
  __shared__ uint32_t bm[kSSGWords];
  __shared__ int pre[kSSGWords];
  const int g = blockIdx.x;
  ssg_mark(rank, nent, nrow, g, bm);
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSSGWords; ++w) {
      pre[w] = t;
      t += __popc(bm[w]);
    }
  }
  const int64_t o = off[g], n = off[g + 1] - o;
  for (int64_t i = threadIdx.x; i < n * kSSG; i += blockDim.x) ucoef[o * kSSG + i] = 0.0;
  __syncthreads();  // zeros stored before the scatter below
  const int r0 = g * kSSG, nr = min(kSSG, nrow - r0);
  for (int i = threadIdx.x; i < nr * nent; i += blockDim.x) {
    const int j = i / nent;
    const int src = rank[(int64_t)r0 * nent + i];
    const int64_t pos = o + pre[src >> 5] + __popc(bm[src >> 5] & ((1u << (src & 31)) - 1u));
    urank[pos] = src;  // every entry of this source writes the same rank
    ucoef[pos * kSSG + j] = coef[(int64_t)r0 * nent + i];
  }
}

// Support-restricted copy of the group lists (sources whose flag is set, in
// order), ccnt[g] their number.  One wave per group.
__global__ void __launch_bounds__(256) k_ssg_compact(const int64_t* __restrict__ off, const int* __restrict__ urank,
                                                     const double* __restrict__ ucoef, int ngroups,
                                                     const uint32_t* __restrict__ src_nz, int* __restrict__ crank,
                                                     double* __restrict__ ccoef, int* __restrict__ ccnt,
                                                     const int* __restrict__ sel) {
  // sel: beside the core path, compact only where the grouped lists are selected
  if (sel && *sel != 0) return;
  const int g = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (g >= ngroups) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t o = off[g];
  const int n = (int)(off[g + 1] - o);
  int kept = 0;
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int k = k0 + lane;
    const int r = k < n ? urank[o + k] : 0;
    const bool keep = k < n && src_nz[r] != 0u;
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int64_t d = o + kept + __popcll(m & below);
      crank[d] = r;
#pragma unroll
      for (int j = 0; j < kSSG; ++j) ccoef[d * kSSG + j] = ucoef[(o + k) * kSSG + j];
    }
    kept += __popcll(m);
  }
  if (lane == 0) ccnt[g] = kept;
}

struct SSGArgs {
  const void* in;           // [nrow][ncol] storage T
  double* out;              // [nrow][ncol] FP64 partial
  const int64_t* off;       // [ngroups + 1] list offsets
  const int* urank;         // union source ranks
  const double* ucoef;      // [.][kSSG] coefficients
  const int* cnt;           // per-group list lengths (support-restricted lists), or null: off differences
  int nrow, ncol, ngroups;
  int ntq;                  // tile groups of kW 64-column tiles (one tile per wave)
  const int* sel;           // with support skipping beside the core path: run only where *sel == 0
};

// out[g*kSSG + j][c] = sum_u ucoef[u][j] in[urank[u]][c] over group g's
// union list.  Each wave owns one group and 64 columns, so the list is
// wave-uniform (scalar loads of ranks and coefficient rows).  A workgroup of
// four waves takes kW neighbouring 64-column tiles of 4 / kW consecutive
// groups.  XCD-aware like k_ss_apply: an XCD's consecutive blocks take
// consecutive groups of one tile group, so that the tile group's slab of the
// input stays in that XCD's L2 as long as it can.
template <typename T, int kW>
__global__ void __launch_bounds__(256) k_ss_apply_g(SSGArgs a) {
  if (a.sel && *a.sel != 0) return;
  constexpr int kGq = 4 / kW;  // groups per workgroup
  const int b = blockIdx.x;
  const int xcd = b & 7, j0 = b >> 3;
  const int ngq = (a.ngroups + kGq - 1) / kGq;
  const int tq = (j0 / ngq) * 8 + xcd;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = (j0 % ngq) * kGq + wv / kW;
  if (tq >= a.ntq || g >= a.ngroups) return;
  const int tile = tq * kW + wv % kW;
  if (tile * 64 >= a.ncol) return;
  const int col = tile * 64 + (threadIdx.x & 63);
  const bool live = col < a.ncol;
  const int colc = live ? col : 0;
  const int64_t o = a.off[g];
  const int n = a.cnt ? __builtin_amdgcn_readfirstlane(a.cnt[g]) : (int)(a.off[g + 1] - o);
  const int* __restrict__ rk = a.urank + o;
  const double* __restrict__ cf = a.ucoef + o * kSSG;
  double acc[kSSG];
#pragma unroll
  for (int j = 0; j < kSSG; ++j) acc[j] = 0.0;
  const T* __restrict__ in = (const T*)a.in;
  int u = 0;
  for (; u + 8 <= n; u += 8) {  // eight independent loads in flight per wave
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = __builtin_amdgcn_readfirstlane(rk[u + i]);
      v[i] = (double)in[(int64_t)r * a.ncol + colc];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < kSSG; ++j) acc[j] = fma(cf[(u + i) * kSSG + j], v[i], acc[j]);
  }
  for (; u < n; ++u) {
    const int r = __builtin_amdgcn_readfirstlane(rk[u]);
    const double v = (double)in[(int64_t)r * a.ncol + colc];
#pragma unroll
    for (int j = 0; j < kSSG; ++j) acc[j] = fma(cf[u * kSSG + j], v, acc[j]);
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < kSSG; ++j) {
    const int r = g * kSSG + j;
    if (r < a.nrow) a.out[(int64_t)r * a.ncol + col] = acc[j];
  }
}

// ---------------------------------------------------------------- mixed rows

struct MixedArgs {
  const void* psi;        // [db][da] storage T
  const double* pa_t;     // alpha same-spin partial, transposed [da][db]
  const double* pb;       // beta same-spin partial [db][da]
  void* sigma;            // [db][da] storage T
  int M, na, nb, da, db;
  const uint32_t* astr;
  const uint32_t* bstr;
  const RankTables* arank;
  const RankTables* brank;
  int nchunk;             // column chunks per beta row
  const uint32_t* row_nz; // support flags of psi's beta rows, or null (every row taken)
  // device-side choice under support skipping: k_mixed_m runs where
  // *sel == 1, k_mixed / k_mixed_c where *sel == 0 (null: no choice)
  const int* sel;
  HamDev H;
};

// sigma[b][a] = pb[b][a] + pa_t[a][b] + (mixed alpha-beta part of H psi)[b][a]
//
// One thread per alpha column.  Its (up to 64) alpha single excitations are
// decoded once into registers as packed entries
//   bits 0..16  LDS address of the source amplitude in the staged row
//   bits 17..28 byte offset of the coefficient s_fab[(pair*2 + O)*2 + sab]
//               (storage-type elements; the table is at LDS address 0),
//               sab = alpha-beta sign (-1)^{popc(abJa & s)}, O = which orbital
//               of the pair is occupied
//   bit  29     single-dressing sign (-1)^{popc(sJ & s)}
// and reused for every staged source row: the workgroup's own beta row (the
// alpha singles' beta-occupation dressing and the alpha-beta diagonal), then
// each beta-single source row (the beta singles' alpha-occupation dressing and
// the alpha-beta doubles).  Coefficient tables with both signs pre-applied sit
// in LDS, so one term is two LDS reads and one FMA.  Unused slots point at the
// zero slot after the row.
// static LDS of k_mixed in one object, coefficient table first: it sits at
// LDS address 0, so the coefficient offsets packed in the entries are
// absolute LDS addresses
template <typename T>
struct MixedLds {
  // [(pid*2+O)*2 + sign], in the storage type: the FP32 path multiplies in
  // FP32 with the coefficient rounded to FP32 either way
  T fab[kMaxPairs * 4];
  double srow[kMaxPairs * 4];  // [(pid*2+O)*2 + sign]
  double dmix[kMaxOrb];
  double bdress[kMaxOrb + 1];  // per stage; [kMaxOrb] = 0 for padded reads
  int2 stage[64];              // per beta single: (source rank, pair | O << 16 | signs << 17)
  int nstage;                  // stages kept (source rows in psi's support)
  int own;                     // the workgroup's own beta row is in psi's support
};

template <typename T>
__global__ void __launch_bounds__(1024) k_mixed(MixedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_row = (T*)smem;  // [da + 1]: the staged row and a zero slot
  if (a.sel && *a.sel != 0) return;
  __shared__ MixedLds<T> L;
  T* const s_fab = L.fab;
  double* const s_srow = L.srow;
  double* const s_dmix = L.dmix;
  double* const s_bdress = L.bdress;
  int2* const s_stage = L.stage;

  const int M = a.M;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, nt = blockDim.x;
  const HamDev& H = a.H;
  // XCD-aware: the column chunks of one beta row run on one XCD
  const int b = blockIdx.x, xcd = b & 7, jj = b >> 3;
  const int brow = (jj / a.nchunk) * 8 + xcd;
  const int chunk = jj % a.nchunk;
  if (brow >= a.db) return;
  const uint32_t bs = a.bstr[brow];
  const int col = chunk * nt + tid;
  const bool live = col < a.da;
  const uint32_t s = live ? a.astr[col] : a.astr[0];

  // Beta-single source rows (stages).  Per stage: the source row's rank, the
  // pair and orientation of the beta excitation and its two signs, tabulated
  // once per workgroup so no dependent lookup precedes a stage's row loads.
  // Rows outside psi's support contribute nothing and are dropped (wave 0,
  // order kept); N_b (M - N_b) <= 64 stages.
  const int nbemp = M - a.nb;
  const int nbs = a.nb * nbemp;
  if (tid < 64) {
    const int jb = tid;
    bool keep = false;
    int2 ent = make_int2(0, 0);
    if (jb < nbs) {
      const int io = jb / nbemp, ie = jb % nbemp;
      uint32_t occ = bs, emp = ~bs & amask;
      for (int j = 0; j < io; ++j) occ &= occ - 1;
      for (int j = 0; j < ie; ++j) emp &= emp - 1;
      const int i = __ffs(occ) - 1, e = __ffs(emp) - 1;
      const int p = min(i, e), q = max(i, e);
      const int pb = pair_id(p, q);
      const uint32_t bs2 = bs ^ (1u << i) ^ (1u << e);
      const uint32_t jsb = H.sJ[kMaxPairs + pb] >> M;
      const uint32_t sgn_s = __popc(jsb & bs) & 1u;
      const uint32_t sgn_ab = __popc((H.abJb[pb] >> M) & bs) & 1u;
      const int r2 = a.brank->lo[bs2 & 255u] + a.brank->hi[(bs2 >> 8) & 255u];
      ent = make_int2(r2, pb | ((i == q) ? 1 << 16 : 0) | (int)(sgn_s << 17) | (int)(sgn_ab << 18));
      keep = !a.row_nz || a.row_nz[r2] != 0u;
    }
    const uint64_t m = __ballot(keep);
    const uint64_t below = (jb == 0) ? 0ull : (~0ull >> (64 - jb));
    if (keep) s_stage[__popcll(m & below)] = ent;
    if (jb == 0) {
      L.nstage = __popcll(m);
      L.own = (!a.row_nz || a.row_nz[brow] != 0u) ? 1 : 0;
    }
  }
  __syncthreads();
  const int nst = L.nstage;
  const bool own = L.own != 0;
  if (nst == 0 && !own) {
    // no source row in psi's support: only the same-spin partials remain
    if (live) {
      const double v = a.pb[(int64_t)brow * a.da + col] + a.pa_t[(int64_t)col * a.db + brow];
      ((T*)a.sigma)[(int64_t)brow * a.da + col] = (T)v;
    }
    return;
  }

  for (int k = tid; k < M; k += nt) {
    double v = 0.0;  // alpha orbital k against the occupied beta orbitals (diagonal)
    uint32_t o = bs;
    while (o) {
      const int l = __ffs(o) - 1;
      o &= o - 1;
      v += H.dC[k * 32 + (l + M)];
    }
    s_dmix[k] = v;
  }
  for (int i = tid; i < kMaxPairs * 2; i += nt) {
    const double* B = H.sB + (size_t)i * 32;  // alpha singles, beta-occupation dressing
    double v = 0.0;
    uint32_t o = bs;
    while (o) {
      const int l = __ffs(o) - 1;
      o &= o - 1;
      v += B[l + M];
    }
    s_srow[2 * i] = v;
    s_srow[2 * i + 1] = -v;
  }
  // packed excitation entries of this thread's alpha string; slots past the
  // string's excitations point at the zero slot s_row[da] (coefficient 0), so
  // the product loops run all 64 slots without predication
  const uint32_t rbase = lds_addr(s_row);  // LDS address of the staged row (below 2^17 with it)
  const uint32_t fbase = lds_addr(s_fab);  // 0: first static LDS object
  uint32_t ex[64];
#pragma unroll
  for (int x = 0; x < 64; ++x) ex[x] = rbase + (uint32_t)a.da * (uint32_t)sizeof(T);
  {
    // every string of the sector has N_a (M - N_a) singles in the same
    // (occupied, empty) order, so the slot counter x and the position ie in
    // the empty list are the same on every lane: each entry goes straight to
    // a fixed register, and the walk to the next occupied orbital is a
    // uniform branch
    const RankTables* R = a.arank;
    const int nemp = M - a.na;
    const int nex = a.na * nemp;
    uint32_t occ = s, emp = 0u;
    int i = 0, ie = nemp;
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      if (x < nex) {
        if (ie == nemp) {
          i = __ffs(occ) - 1;
          occ &= occ - 1;
          emp = ~s & amask;
          ie = 0;
        }
        const int e = __ffs(emp) - 1;
        emp &= emp - 1;
        ++ie;
        const int p = min(i, e), q = max(i, e);
        const int pid = pair_id(p, q);
        const uint32_t t2 = s ^ (1u << i) ^ (1u << e);
        const uint32_t r2 = (uint32_t)(R->lo[t2 & 255u] + R->hi[(t2 >> 8) & 255u]);
        const uint32_t sab = __popc(H.abJa[pid] & s) & 1u;
        const uint32_t ssg = __popc(H.sJ[pid] & s) & 1u;
        const uint32_t O = (i == q) ? 1u : 0u;
        // LDS byte offsets: the source amplitude (bits 0..16) and the
        // coefficient s_fab[(pair*2 + O)*2 + sab] (bits 17..28); bit 29 is
        // the sign of the singles' dressing
        ex[x] = (rbase + r2 * (uint32_t)sizeof(T)) |
                (((((uint32_t)pid * 2u + O) * 2u + sab) * (uint32_t)sizeof(T)) << 17) | (ssg << 29);
      }
    }
  }
  const T* psi = (const T*)a.psi;
  if (tid == 0) s_row[a.da] = T(0);
  double acc = 0.0;
  // (1) own row: alpha-beta diagonal and alpha singles' beta dressing
  if (own) {
    stage_row_lds(s_row, psi + (int64_t)brow * a.da, a.da * (int)sizeof(T), tid, nt);
    __syncthreads();
    double v = 0.0;
    uint32_t o = s;
    while (o) {
      const int i = __ffs(o) - 1;
      o &= o - 1;
      v += s_dmix[i];
    }
    acc += Acc<T>::prod(v, s_row[live ? col : 0]);
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      const uint32_t e = ex[x];
      const int fi = (int)(((((e >> 17) & 0xfffu) / (uint32_t)sizeof(T)) & ~1u) | ((e >> 29) & 1u));
      acc += Acc<T>::prod(s_srow[fi], lds_load<T>(e & 0x1ffffu));
    }
    asm volatile("" : "+v"(acc));  // finish the products here, not after the table loop below
  }

  // (2) the kept beta-single source rows
  // LDS addresses of s_bdress entries of this thread's occupied orbitals,
  // padded with the zero entry, for the per-stage dressing sum
  uint32_t occ_off[16];
  {
    const uint32_t dbase = lds_addr(s_bdress);
    const uint32_t zero = lds_addr(&s_bdress[kMaxOrb]);
    uint32_t o = s;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      occ_off[j] = o ? dbase + (uint32_t)(__ffs(o) - 1) * 8u : zero;
      o &= o - 1;
    }
  }
  if (tid == 0) s_bdress[kMaxOrb] = 0.0;
  const int occ_groups = (__popc(s) + 7) >> 3;  // same for every thread
  for (int jb = 0; jb < nst; ++jb) {
    // the entries are opaque to the optimiser here: otherwise it hoists the
    // 128 addresses derived from them out of the loop and spills
#pragma unroll
    for (int x = 0; x < 64; ++x) asm volatile("" : "+v"(ex[x]));
    __syncthreads();
    // the stage's coefficient (alpha excitation tid) and dressing (orbital
    // tid) are loaded first and stored after the row copy is issued, so one
    // wait covers all three
    const int info = s_stage[jb].y;
    const int pb = info & 0xffff, Ob = (info >> 16) & 1;
    double f_ld = 0.0, d_ld = 0.0;
    if (tid < kMaxPairs * 2)
      f_ld = H.abF[((size_t)(tid >> 1) * kMaxPairs + pb) * 4 + (tid & 1) * 2 + Ob];
    if (tid < M) d_ld = H.sB[(size_t)((kMaxPairs + pb) * 2 + Ob) * 32 + tid];
    stage_row_lds(s_row, psi + (int64_t)s_stage[jb].x * a.da, a.da * (int)sizeof(T), tid, nt);
    asm volatile("" ::: "memory");
    if (tid < kMaxPairs * 2) {
      const double f = ((info >> 18) & 1) ? -f_ld : f_ld;
      s_fab[2 * tid] = (T)f;
      s_fab[2 * tid + 1] = (T)(-f);
    }
    if (tid < M) s_bdress[tid] = ((info >> 17) & 1) ? -d_ld : d_ld;
    for (int x = tid + nt; x < kMaxPairs * 2; x += nt) {  // only when nt < 240
      const int pa = x >> 1, Oa = x & 1;
      const double f0 = H.abF[((size_t)pa * kMaxPairs + pb) * 4 + Oa * 2 + Ob];
      const double f = ((info >> 18) & 1) ? -f0 : f0;
      s_fab[2 * x] = (T)f;
      s_fab[2 * x + 1] = (T)(-f);
    }
    __syncthreads();
    double dr = 0.0;
    {
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < occ_groups) {
          double v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = lds_load<double>(occ_off[g * 8 + j]);
#pragma unroll
          for (int j = 0; j < 8; ++j) dr += v[j];
        }
    }
    double sum = Acc<T>::prod(dr, s_row[live ? col : 0]);
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      const uint32_t e2 = ex[x];
      sum += Acc<T>::prod(lds_load<T>(fbase + ((e2 >> 17) & 0xfffu)), lds_load<T>(e2 & 0x1ffffu));
    }
    acc += sum;
    asm volatile("" : "+v"(acc));
  }

  // (3) combine with the two same-spin partials and store
  if (live) {
    const double v = acc + a.pb[(int64_t)brow * a.da + col] + a.pa_t[(int64_t)col * a.db + brow];
    ((T*)a.sigma)[(int64_t)brow * a.da + col] = (T)v;
  }
}

// k_mixed for FP64 with compact, double-buffered staging: 768-column chunks
// (at 16 orbitals and 8 electrons at most 4083 blocks, 52% of a row) stage only the 16-byte blocks of a source row their columns reach (the
// chunk's list from the compact tables), into buffers alternating between
// LDS byte offsets 0 and kCBuf1 of the dynamic area; the coefficient and
// dressing tables of a stage alternate with them, so that the next source
// row's copy and table fill overlap this row's products.  Per output the
// products, and the order they are summed in, are those of k_mixed: sigma is
// the same bit for bit.
struct MixedLdsC {
  double fab[2][kMaxPairs * 4];   // per buffer: [(pid*2+O)*2 + sign]
  double srow[kMaxPairs * 4];     // [(pid*2+O)*2 + sign]
  double dmix[kMaxOrb];
  double bdress[2][kMaxOrb + 1];  // per buffer; [kMaxOrb] = 0 for padded reads
  int2 stage[64];
  int nstage;
  int own;
};
constexpr uint32_t kFab1 = kMaxPairs * 4 * 8;  // byte offset of fab[1] from fab[0]
constexpr uint32_t kBd1 = (kMaxOrb + 1) * 8;   // byte offset of bdress[1] from bdress[0]

__global__ void __launch_bounds__(768) k_mixed_c(MixedArgs a, const uint16_t* __restrict__ bpos,
                                                 const uint16_t* __restrict__ blist, const int* __restrict__ nblk_c,
                                                 int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ MixedLdsC L;
  if (a.sel && *a.sel != 0) return;
  const int M = a.M;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, nt = blockDim.x;
  const HamDev& H = a.H;
  const int b = blockIdx.x, xcd = b & 7, jj = b >> 3;
  const int brow = (jj / a.nchunk) * 8 + xcd;
  const int chunk = jj % a.nchunk;
  if (brow >= a.db) return;
  const uint32_t bs = a.bstr[brow];
  const int col = chunk * nt + tid;
  const bool live = col < a.da;
  const uint32_t s = live ? a.astr[col] : a.astr[0];

  // stage table, as in k_mixed
  const int nbemp = M - a.nb;
  const int nbs = a.nb * nbemp;
  if (tid < 64) {
    const int jb = tid;
    bool keep = false;
    int2 ent = make_int2(0, 0);
    if (jb < nbs) {
      const int io = jb / nbemp, ie = jb % nbemp;
      uint32_t occ = bs, emp = ~bs & amask;
      for (int j = 0; j < io; ++j) occ &= occ - 1;
      for (int j = 0; j < ie; ++j) emp &= emp - 1;
      const int i = __ffs(occ) - 1, e = __ffs(emp) - 1;
      const int p = min(i, e), q = max(i, e);
      const int pb = pair_id(p, q);
      const uint32_t bs2 = bs ^ (1u << i) ^ (1u << e);
      const uint32_t jsb = H.sJ[kMaxPairs + pb] >> M;
      const uint32_t sgn_s = __popc(jsb & bs) & 1u;
      const uint32_t sgn_ab = __popc((H.abJb[pb] >> M) & bs) & 1u;
      const int r2 = a.brank->lo[bs2 & 255u] + a.brank->hi[(bs2 >> 8) & 255u];
      ent = make_int2(r2, pb | ((i == q) ? 1 << 16 : 0) | (int)(sgn_s << 17) | (int)(sgn_ab << 18));
      keep = !a.row_nz || a.row_nz[r2] != 0u;
    }
    const uint64_t m = __ballot(keep);
    const uint64_t below = (jb == 0) ? 0ull : (~0ull >> (64 - jb));
    if (keep) L.stage[__popcll(m & below)] = ent;
    if (jb == 0) {
      L.nstage = __popcll(m);
      L.own = (!a.row_nz || a.row_nz[brow] != 0u) ? 1 : 0;
    }
  }
  __syncthreads();
  const int nst = L.nstage;
  const bool own = L.own != 0;
  if (nst == 0 && !own) {
    if (live) {
      const double v = a.pb[(int64_t)brow * a.da + col] + a.pa_t[(int64_t)col * a.db + brow];
      ((double*)a.sigma)[(int64_t)brow * a.da + col] = v;
    }
    return;
  }
  for (int k = tid; k < M; k += nt) {
    double v = 0.0;
    uint32_t o = bs;
    while (o) {
      const int l = __ffs(o) - 1;
      o &= o - 1;
      v += H.dC[k * 32 + (l + M)];
    }
    L.dmix[k] = v;
  }
  for (int i = tid; i < kMaxPairs * 2; i += nt) {
    const double* B = H.sB + (size_t)i * 32;
    double v = 0.0;
    uint32_t o = bs;
    while (o) {
      const int l = __ffs(o) - 1;
      o &= o - 1;
      v += B[l + M];
    }
    L.srow[2 * i] = v;
    L.srow[2 * i + 1] = -v;
  }
  // compact positions: block b of a row sits at byte 16 * bp[b] of a buffer
  const uint32_t rbase = lds_addr(smem);
  const int nbk = nblk_c[chunk];
  const uint16_t* bp = bpos + (int64_t)chunk * nblk;
  const uint32_t zslot = rbase + (uint32_t)nbk * 16u;
  const uint32_t fbase = lds_addr(&L.fab[0][0]);
  uint32_t ex[64];
#pragma unroll
  for (int x = 0; x < 64; ++x) ex[x] = zslot;
  {
    const RankTables* R = a.arank;
    const int nemp = M - a.na;
    const int nex = a.na * nemp;
    uint32_t occ = s, emp = 0u;
    int i = 0, ie = nemp;
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      if (x < nex) {
        if (ie == nemp) {
          i = __ffs(occ) - 1;
          occ &= occ - 1;
          emp = ~s & amask;
          ie = 0;
        }
        const int e = __ffs(emp) - 1;
        emp &= emp - 1;
        ++ie;
        const int p = min(i, e), q = max(i, e);
        const int pid = pair_id(p, q);
        const uint32_t t2 = s ^ (1u << i) ^ (1u << e);
        const uint32_t r2 = (uint32_t)(R->lo[t2 & 255u] + R->hi[(t2 >> 8) & 255u]);
        const uint32_t sab = __popc(H.abJa[pid] & s) & 1u;
        const uint32_t ssg = __popc(H.sJ[pid] & s) & 1u;
        const uint32_t O = (i == q) ? 1u : 0u;
        const uint32_t amp = live ? rbase + (uint32_t)bp[r2 >> 1] * 16u + (r2 & 1u) * 8u : zslot;
        ex[x] = amp | ((((uint32_t)pid * 2u + O) * 2u + sab) * 8u << 17) | (ssg << 29);
      }
    }
  }
  const uint32_t ocol = live ? rbase + (uint32_t)bp[col >> 1] * 16u + ((uint32_t)col & 1u) * 8u : zslot;
  int blk[kCPerThread];
#pragma unroll
  for (int k = 0; k < kCPerThread; ++k) {
    const int i = k * nt + tid;
    blk[k] = i < nbk ? (int)blist[(int64_t)chunk * kCMaxBlk + i] : 0;
  }
  uint32_t occ_off[16];
  {
    const uint32_t dbase = lds_addr(&L.bdress[0][0]);
    const uint32_t zero = lds_addr(&L.bdress[0][kMaxOrb]);
    uint32_t o = s;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      occ_off[j] = o ? dbase + (uint32_t)(__ffs(o) - 1) * 8u : zero;
      o &= o - 1;
    }
  }
  const int occ_groups = (__popc(s) + 7) >> 3;
  if (tid == 0) {
    *(__attribute__((address_space(3))) double*)(uintptr_t)zslot = 0.0;
    *(__attribute__((address_space(3))) double*)(uintptr_t)(zslot + kCBuf1) = 0.0;
    L.bdress[0][kMaxOrb] = 0.0;
    L.bdress[1][kMaxOrb] = 0.0;
  }
  const double* psi = (const double*)a.psi;
  const int ownoff = own ? 1 : 0;
  const int nitems = ownoff + nst;  // item 0 the own row when kept, then the stages
  auto src_of = [&](int it) -> int { return (own && it == 0) ? brow : L.stage[it - ownoff].x; };
  // coefficient and dressing values of stage item `it`, thread tid's entries
  auto load_coef = [&](int it, double& f_ld, double& d_ld) {
    const int info = L.stage[it - ownoff].y;
    const int pb = info & 0xffff, Ob = (info >> 16) & 1;
    f_ld = 0.0;
    d_ld = 0.0;
    if (tid < kMaxPairs * 2) f_ld = H.abF[((size_t)(tid >> 1) * kMaxPairs + pb) * 4 + (tid & 1) * 2 + Ob];
    if (tid < M) d_ld = H.sB[(size_t)((kMaxPairs + pb) * 2 + Ob) * 32 + tid];
  };
  auto write_coef = [&](int P, int it, double f_ld, double d_ld) {
    const int info = L.stage[it - ownoff].y;
    if (tid < kMaxPairs * 2) {
      const double f = ((info >> 18) & 1) ? -f_ld : f_ld;
      L.fab[P][2 * tid] = f;
      L.fab[P][2 * tid + 1] = -f;
    }
    if (tid < M) L.bdress[P][tid] = ((info >> 17) & 1) ? -d_ld : d_ld;
  };
  double acc = 0.0;
  // prologue: item 0's row into buffer 0 (and its tables, for a stage)
  stage_blocks(rbase, psi + (int64_t)src_of(0) * a.da, blk, nbk, tid, nt);
  if (!own) {
    double f_ld, d_ld;
    load_coef(0, f_ld, d_ld);
    write_coef(0, 0, f_ld, d_ld);
  }
  auto step = [&](auto pc, auto ownc, int it) {
    constexpr int P = decltype(pc)::value;
    constexpr bool kOwn = decltype(ownc)::value;
    constexpr uint32_t kBuf = P ? kCBuf1 : 0u;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // item it staged and its tables written; reads of the other buffer done
    const bool nxt = it + 1 < nitems;
    double f_ld = 0.0, d_ld = 0.0;
    if (nxt) {
      load_coef(it + 1, f_ld, d_ld);
      stage_blocks(rbase + (P ? 0u : kCBuf1), psi + (int64_t)src_of(it + 1) * a.da, blk, nbk, tid, nt);
    }
    if (kOwn) {
      // alpha-beta diagonal and the alpha singles' beta dressing (buffer 0)
      double v = 0.0;
      uint32_t o = s;
      while (o) {
        const int i = __ffs(o) - 1;
        o &= o - 1;
        v += L.dmix[i];
      }
      acc += v * lds_load<double>(ocol);
#pragma unroll
      for (int x = 0; x < 64; ++x) {
        const uint32_t e = ex[x];
        const int fi = (int)(((((e >> 17) & 0xfffu) / 8u) & ~1u) | ((e >> 29) & 1u));
        acc += L.srow[fi] * lds_load<double>(e & 0x1ffffu);
      }
      asm volatile("" : "+v"(acc));
    } else {
#pragma unroll
      for (int x = 0; x < 64; ++x) asm volatile("" : "+v"(ex[x]));
      double dr = 0.0;
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < occ_groups) {
          double v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = lds_load<double>(occ_off[g * 8 + j] + (P ? kBd1 : 0u));
#pragma unroll
          for (int j = 0; j < 8; ++j) dr += v[j];
        }
      double sum = dr * lds_load<double>(ocol + kBuf);
#pragma unroll
      for (int x = 0; x < 64; ++x) {
        const uint32_t e2 = ex[x];
        sum += lds_load<double>(fbase + ((e2 >> 17) & 0xfffu) + (P ? kFab1 : 0u)) *
               lds_load<double>((e2 & 0x1ffffu) + kBuf);
      }
      acc += sum;
      asm volatile("" : "+v"(acc));
    }
    if (nxt) write_coef(P ? 0 : 1, it + 1, f_ld, d_ld);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using BF = std::integral_constant<bool, false>;
  using BT = std::integral_constant<bool, true>;
  int it = 0;
  if (own) step(I0(), BT(), it++);
  if ((it & 1) && it < nitems) step(I1(), BF(), it++);
  for (; it + 1 < nitems; it += 2) {
    step(I0(), BF(), it);
    step(I1(), BF(), it + 1);
  }
  if (it < nitems) step(I0(), BF(), it);

  if (live) {
    const double v = acc + a.pb[(int64_t)brow * a.da + col] + a.pa_t[(int64_t)col * a.db + brow];
    ((double*)a.sigma)[(int64_t)brow * a.da + col] = v;
  }
}

// ------------------------------------------------ mixed pass on matrix cores
//
// The alpha-beta part of one beta row I_b as dense products.  Stage the row's
// kept beta-single sources J_k (k < K <= 64) as a K x D_a matrix
// P[k][t] = psi[J_k][t].  An alpha single takes source string t to output
// string s = t - e + i (e occupied in t, i empty in t), so every alpha-beta
// double of the row is
//   sigma[I_b][s] += (-1)^{popc(abJa[(i,e)] & s)} Z_e[i][t],
//   Z_e[i][t] = sum_k A_e[i][k] P[k][t],
//   A_e[i][k] = (beta sign of k) abF[(i,e)][pair of k][i > e][orientation of k],
// and the beta singles' alpha-occupation dressing is row i = e of the same
// product, A_e[e][k] being the dressing coefficient of orbital e for stage k
// (target s = t).  For one orbital e that is a (16 x K) x (K x |{t : e in t}|)
// product on v_mfma_f64_16x16x4_f64: wave e keeps A_e in registers (one A
// operand per 4 stages) and takes a chunk's columns with e occupied, 16 at a
// time, as B operands from LDS (element q of lane l holds row (l >> 4) + 4q
// of Z_e, column l & 15).  The own row (the alpha singles' beta dressing and
// the alpha-beta diagonal) is a rank-one term on the same targets.  Each
// target is added to the output row, held whole in LDS, with ds_add_f64.
// Which columns a wave takes and where and with which signs each element
// lands depend on the alpha strings only: k_mm_tables lists them once per
// Hamiltonian.  The waves' additions land in no fixed order, so this form
// reproduces sigma to rounding, not bit for bit (k_mixed and k_mixed_c are
// the bitwise-reproducible forms).  Products and sums in FP64 for either
// storage type.
constexpr int kMMSeg = 16;                 // columns per segment (one 128-byte line at FP64)
constexpr int kMMSegs = 3;                 // segments per chunk, from three regions of the alpha space
constexpr int kMMCols = kMMSeg * kMMSegs;  // source columns per chunk
constexpr int kMMTiles = (kMMCols + 15) / 16;
constexpr uint32_t kMMNone = 0x3fffu;      // target code: no element
// A chunk takes segment c of each of the kMMSegs equal regions of the alpha
// columns, so that every chunk mixes strings of all occupations and the
// 16 waves' (orbitals') column counts stay close; chunks alternate between
// two buffers filled by direct global->LDS copies.
__host__ __device__ inline int mm_column(int c, int l, int qr) {
  return (l / kMMSeg) * qr + c * kMMSeg + l % kMMSeg;
}

// The row-independent tables: one wave per (chunk c, orbital e).  Its
// columns with e occupied in chunk order fill 16-slot tiles; lane
// l = 16 g + u of tile j takes slot 16 j + u and rows i = g + 4q.
__global__ void __launch_bounds__(64) k_mm_tables(int M, int da, int qr, const uint32_t* __restrict__ astr,
                                                  const RankTables* __restrict__ arank,
                                                  const uint32_t* __restrict__ abJa, const uint32_t* __restrict__ sJ,
                                                  uint32_t* __restrict__ ent, uint64_t* __restrict__ code,
                                                  uint8_t* __restrict__ nt) {
  __shared__ uint32_t lst[64];
  const int ce = blockIdx.x, c = ce >> 4, e = ce & 15, lane = threadIdx.x;
  const int g = mm_column(c, lane, qr);
  const uint32_t t0 = (lane < kMMCols && g < da) ? astr[g] : 0u;
  const bool bit = e < M && ((t0 >> e) & 1u);
  const uint64_t m = __ballot(bit);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (bit) lst[__popcll(m & below)] = (uint32_t)lane | (t0 << 8);
  __syncthreads();
  const int n = __popcll(m);
  if (lane == 0) nt[ce] = (uint8_t)((n + 15) >> 4);
  for (int j = 0; j < kMMTiles; ++j) {
    const int slot = 16 * j + (lane & 15);
    const bool valid = slot < n;
    const uint32_t en = valid ? lst[slot] : 0u;
    const uint32_t t = en >> 8;
    const size_t tile = (size_t)ce * kMMTiles + j;
    if (lane < 16) ent[tile * 16 + lane] = en;
    uint64_t cw = 0;
    for (int q = 0; q < 4; ++q) {
      const int i = (lane >> 4) + 4 * q;
      uint32_t cq = kMMNone;
      if (valid && i < M && (i == e || !((t >> i) & 1u))) {
        const uint32_t s2 = (i == e) ? t : t ^ (1u << e) ^ (1u << i);
        const uint32_t r = (uint32_t)(arank->lo[s2 & 255u] + arank->hi[(s2 >> 8) & 255u]);
        uint32_t sab = 0u, ssg = 0u;
        if (i != e) {
          const int pid = pair_id(min(i, e), max(i, e));
          sab = __popc(abJa[pid] & s2) & 1u;
          ssg = __popc(sJ[pid] & s2) & 1u;
        }
        cq = r | (sab << 14) | (ssg << 15);
      }
      cw |= (uint64_t)cq << (16 * q);
    }
    code[tile * 64 + lane] = cw;
  }
}

template <typename T>
struct MixedMMLds {
  T P[2][65][kMMCols];  // rows < 64: kept beta-single sources (zero past them); row 64: own row
  int2 stage[64];
  int nstage;
  int own;
};
constexpr size_t kMMLdsMax = 160 * 1024;  // LDS per workgroup

// qr: columns per region (a multiple of kMMSeg), nch = qr / kMMSeg chunks;
// kVec: rows start 16-byte aligned (16-byte copies, else 4-byte)
template <typename T, int kVec>
__global__ void __launch_bounds__(1024) k_mixed_m(MixedArgs a, const uint32_t* __restrict__ ment,
                                                  const uint64_t* __restrict__ mcode, const uint8_t* __restrict__ mnt,
                                                  int qr, int nch) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) MixedMMLds<T> L;
  if (a.sel && *a.sel != 1) return;
  double* sig = (double*)smem;  // [da]: the row's alpha-beta part
  const int M = a.M, da = a.da;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const HamDev& H = a.H;
  const int brow = blockIdx.x;
  const uint32_t bs = a.bstr[brow];

  // stage table, as in k_mixed
  const int nbemp = M - a.nb;
  const int nbs = a.nb * nbemp;
  if (tid < 64) {
    const int jb = tid;
    bool keep = false;
    int2 ent = make_int2(0, 0);
    if (jb < nbs) {
      const int io = jb / nbemp, ie = jb % nbemp;
      uint32_t occ = bs, emp = ~bs & amask;
      for (int j = 0; j < io; ++j) occ &= occ - 1;
      for (int j = 0; j < ie; ++j) emp &= emp - 1;
      const int i = __ffs(occ) - 1, e = __ffs(emp) - 1;
      const int p = min(i, e), q = max(i, e);
      const int pb = pair_id(p, q);
      const uint32_t bs2 = bs ^ (1u << i) ^ (1u << e);
      const uint32_t jsb = H.sJ[kMaxPairs + pb] >> M;
      const uint32_t sgn_s = __popc(jsb & bs) & 1u;
      const uint32_t sgn_ab = __popc((H.abJb[pb] >> M) & bs) & 1u;
      const int r2 = a.brank->lo[bs2 & 255u] + a.brank->hi[(bs2 >> 8) & 255u];
      ent = make_int2(r2, pb | ((i == q) ? 1 << 16 : 0) | (int)(sgn_s << 17) | (int)(sgn_ab << 18));
      keep = !a.row_nz || a.row_nz[r2] != 0u;
    }
    const uint64_t m = __ballot(keep);
    const uint64_t below = (jb == 0) ? 0ull : (~0ull >> (64 - jb));
    if (keep) L.stage[__popcll(m & below)] = ent;
    if (jb == 0) {
      L.nstage = __popcll(m);
      L.own = (!a.row_nz || a.row_nz[brow] != 0u) ? 1 : 0;
    }
  }
  __syncthreads();
  const int nst = L.nstage;
  const bool own = L.own != 0;
  if (nst == 0 && !own) {
    for (int c = tid; c < da; c += 1024) {
      const double v = a.pb[(int64_t)brow * da + c] + a.pa_t[(int64_t)c * a.db + brow];
      ((T*)a.sigma)[(int64_t)brow * da + c] = (T)v;
    }
    return;
  }
  for (int c = tid; c < da; c += 1024) sig[c] = 0.0;
  // source rows past the kept ones stay zero in both buffers, and so does
  // the own row when it is not taken
  for (int x = tid; x < 2 * 65 * kMMCols; x += 1024) {
    const int r = (x / kMMCols) % 65;
    if ((r >= nst && r < 64) || (r == 64 && !own)) (&L.P[0][0][0])[x] = T(0);
  }
  const int nks = (nst + 3) >> 2;  // MFMA steps of 4 stages

  // wave w: alpha orbital e = w; its A operands (lane l: row l & 15, stage
  // 4 step + (l >> 4))
  const int e = w;
  const bool ew = e < M;
  double areg[16];
  {
    const int i = lane & 15;
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int k = 4 * st + (lane >> 4);
      double v = 0.0;
      if (ew && i < M && k < nst) {
        const int info = L.stage[k].y;
        const int pb = info & 0xffff, Ob = (info >> 16) & 1;
        if (i == e) {
          const double d = H.sB[(size_t)((kMaxPairs + pb) * 2 + Ob) * 32 + e];
          v = ((info >> 17) & 1) ? -d : d;
        } else {
          const int pid = pair_id(min(i, e), max(i, e));
          const double f = H.abF[((size_t)pid * kMaxPairs + pb) * 4 + (i > e ? 2 : 0) + Ob];
          v = ((info >> 18) & 1) ? -f : f;
        }
      }
      areg[st] = v;
    }
  }
  // the own row's coefficient per output element q of a lane (row
  // i = (l >> 4) + 4q of Z_e): the alpha single's beta dressing of the pair
  // (i, e), for i = e the alpha-beta diagonal of e
  double cown[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = (lane >> 4) + 4 * q;
    double v = 0.0;
    if (ew && own && i < M) {
      uint32_t o = bs;
      if (i == e) {
        while (o) {
          const int l = __ffs(o) - 1;
          o &= o - 1;
          v += H.dC[e * 32 + (l + M)];
        }
      } else {
        const double* B = H.sB + (size_t)(pair_id(min(i, e), max(i, e)) * 2 + (i > e ? 1 : 0)) * 32;
        while (o) {
          const int l = __ffs(o) - 1;
          o &= o - 1;
          v += B[l + M];
        }
      }
    }
    cown[q] = v;
  }
  // the set-up loads complete here, not behind the chunk loop's copies
#pragma unroll
  for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(cown[q]));
#pragma unroll
  for (int st = 0; st < 16; ++st) asm volatile("" : "+v"(areg[st]));

  // chunk c into buffer bf: piece p (kPB bytes) of the 65 x kMMCols buffer
  // from row p / kPPR; lane l of a wave writes its piece at the wave's base +
  // kPB l.  A thread's pieces are p = 1024 it + 64 w + lane; their source
  // addresses at chunk 0, set once, advance by kMMSeg columns per chunk.
  constexpr int kPB = kVec ? 16 : 4;
  constexpr int kPPR = kMMCols * (int)sizeof(T) / kPB;  // pieces per row
  constexpr int kNP = 65 * kPPR;                       // pieces per buffer
  constexpr int kIt = (kNP + 1023) / 1024;
  // (with more than 4 pieces per thread, the FP64 4-byte form, the
  // addresses are formed per chunk instead)
  constexpr int kPre = kIt <= 4 ? kIt : 0;
  const T* psi = (const T*)a.psi;
  auto piece = [&](int it, int& g, uint32_t& off) {
    const int p = it * 1024 + w * 64 + lane;
    const int row = p / kPPR;
    const int lb = (p % kPPR) * kPB;  // byte in the row
    g = mm_column(0, lb / (int)sizeof(T), qr);
    const bool ok = p < kNP && (row < nst || (row == 64 && own));
    const int src = row == 64 ? brow : (row < nst ? L.stage[row].x : 0);
    off = (uint32_t)((int64_t)src * da + g);
    if (!ok) g = -1;
  };
  uint32_t off0[kPre > 0 ? kPre : 1];  // source element at chunk 0 (the state has < 2^32 elements wherever the row fits LDS)
  int g0[kPre > 0 ? kPre : 1];         // column of the piece at chunk 0, -1 when it is not copied
#pragma unroll
  for (int it = 0; it < kPre; ++it) piece(it, g0[it], off0[it]);
  auto copy = [&](uint32_t dst, int base, int c, int g, uint32_t off) {
    if (g >= 0 && g + c * kMMSeg < da) {
      const int lb = ((base + lane) % kPPR) * kPB;
      const char* gp = (const char*)(psi + off + (uint32_t)c * kMMSeg) + lb % (int)sizeof(T);
      if (kVec)
        dma16(dst, gp);
      else
        dma4(dst, gp);
    }
  };
  auto issue = [&](int c, int bf) {
    const uint32_t buf = lds_addr(&L.P[bf][0][0]);
    if constexpr (kPre > 0) {
#pragma unroll
      for (int it = 0; it < kPre; ++it) {
        const int base = it * 1024 + w * 64;  // wave-uniform
        if (base < kNP)
          copy((uint32_t)__builtin_amdgcn_readfirstlane(buf + (uint32_t)base * (uint32_t)kPB), base, c, g0[it],
               off0[it]);
      }
    } else {
#pragma unroll 1
      for (int it = 0; it < kIt; ++it) {
        const int base = it * 1024 + w * 64;
        if (base < kNP) {
          int g;
          uint32_t off;
          piece(it, g, off);
          copy((uint32_t)__builtin_amdgcn_readfirstlane(buf + (uint32_t)base * (uint32_t)kPB), base, c, g, off);
        }
      }
    }
  };
  // the wave's tables of chunk c
  int ntn = 0;
  uint32_t entn[kMMTiles];
  uint64_t coden[kMMTiles];
  auto tables = [&](int c) {
    const size_t ce = (size_t)c * 16 + e;
    ntn = ew ? __builtin_amdgcn_readfirstlane((int)mnt[ce]) : 0;
#pragma unroll
    for (int j = 0; j < kMMTiles; ++j) {
      entn[j] = 0u;
      coden[j] = ~0ull;
      if (j < ntn) {
        entn[j] = ment[(ce * kMMTiles + j) * 16 + (lane & 15)];
        coden[j] = mcode[(ce * kMMTiles + j) * 64 + lane];
      }
    }
  };

  const uint32_t pbase0 = lds_addr(&L.P[0][lane >> 4][0]);
  constexpr uint32_t kBufBytes = 65u * kMMCols * sizeof(T);
  constexpr uint32_t kStep = 4u * kMMCols * sizeof(T);  // 4 stages
  // Z_e of one tile (column col of buffer pbc)
  auto products = [&](uint32_t pbc, uint32_t col) -> f64x4 {
    const uint32_t pb = pbc + col * (uint32_t)sizeof(T);
    f64x4 z0 = {0.0, 0.0, 0.0, 0.0}, z1 = {0.0, 0.0, 0.0, 0.0};
    if (nks == 16) {
      // every stage kept: all B operands read, then the products
#pragma unroll
      for (int h = 0; h < 16; h += 8) {
        // eight B operands read, then their products
        double bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = (double)lds_load<T>(pb + (h + u) * kStep);
        asm volatile("" ::"v"(bv[0]), "v"(bv[1]), "v"(bv[2]), "v"(bv[3]), "v"(bv[4]), "v"(bv[5]), "v"(bv[6]),
                     "v"(bv[7]));
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[h + u], bv[u], z0, 0, 0, 0);
          z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[h + u + 1], bv[u + 1], z1, 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int st = 0; st < 16; st += 2) {
        if (st < nks)
          z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[st], (double)lds_load<T>(pb + st * kStep), z0, 0, 0, 0);
        if (st + 1 < nks)
          z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(areg[st + 1], (double)lds_load<T>(pb + (st + 1) * kStep), z1, 0,
                                                    0, 0);
      }
    }
    return z0 + z1;
  };
  // each element of the tile to its target in the row
  auto scatter = [&](uint32_t obase, uint32_t col, uint64_t cw, const f64x4& z) {
    const double pown = (double)lds_load<T>(obase + col * (uint32_t)sizeof(T));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t cq = (uint32_t)(cw >> (16 * q)) & 0xffffu;
      const uint32_t r = cq & 0x3fffu;
      const double zz = (cq & 0x4000u) ? -z[q] : z[q];
      const double cc = (cq & 0x8000u) ? -cown[q] : cown[q];
      if (r != kMMNone) atomicAdd(&sig[r], zz + cc * pown);
    }
  };

  tables(0);
  issue(0, 0);
  for (int c = 0; c < nch; ++c) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();  // chunk c in its buffer; every wave done with chunk c - 1
    const int ntile = ntn;
    uint32_t ent[kMMTiles];
    uint64_t code[kMMTiles];
#pragma unroll
    for (int j = 0; j < kMMTiles; ++j) {
      ent[j] = entn[j];
      code[j] = coden[j];
    }
    const uint32_t pbc = pbase0 + (uint32_t)(c & 1) * kBufBytes;
    const uint32_t obase = lds_addr(&L.P[c & 1][64][0]);
    // the first tile's products run while the next chunk's tables and
    // copies go out
    f64x4 z = {0.0, 0.0, 0.0, 0.0};
    if (ntile > 0) z = products(pbc, ent[0] & 63u);
    if (c + 1 < nch) {
      tables(c + 1);
      issue(c + 1, (c + 1) & 1);
    }
    if (ntile > 0) scatter(obase, ent[0] & 63u, code[0], z);
#pragma unroll
    for (int j = 1; j < kMMTiles; ++j) {
      if (j < ntile) {
        const f64x4 zj = products(pbc, ent[j] & 63u);
        scatter(obase, ent[j] & 63u, code[j], zj);
      }
    }
  }
  __syncthreads();  // every addition into the row done
  for (int c = tid; c < da; c += 1024) {
    const double v = sig[c] + a.pb[(int64_t)brow * da + c] + a.pa_t[(int64_t)c * a.db + brow];
    ((T*)a.sigma)[(int64_t)brow * da + c] = (T)v;
  }
}

// ---------------------------------------------------------------- generic

struct GenericArgs {
  const void* psi;
  void* sigma;
  int M, na, nb, da;
  int64_t dim;
  const uint32_t* astr;
  const uint32_t* bstr;
  const RankTables* arank;
  const RankTables* brank;
  int64_t ngroup;
  const uint32_t* gx;
  const int64_t* goff;
  const uint32_t* tz;
  const double* tc;
};

// One thread per output amplitude, every X-group in turn (any real Pauli sum).
template <typename T>
__global__ void k_generic(GenericArgs a) {
  int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= a.dim) return;
  const uint32_t amask = (1u << a.M) - 1u;
  const uint32_t bd = a.astr[d % a.da] | (a.bstr[d / a.da] << a.M);
  const T* psi = (const T*)a.psi;
  double acc = 0.0;
  for (int64_t g = 0; g < a.ngroup; ++g) {
    const uint32_t b = bd ^ a.gx[g];
    const uint32_t ba = b & amask, bb = b >> a.M;
    if (__popc(ba) != a.na || __popc(bb) != a.nb) continue;
    const int64_t src = (int64_t)(a.brank->lo[bb & 255u] + a.brank->hi[(bb >> 8) & 255u]) * a.da +
                        (a.arank->lo[ba & 255u] + a.arank->hi[(ba >> 8) & 255u]);
    double cf = 0.0;
    for (int64_t t = a.goff[g]; t < a.goff[g + 1]; ++t) cf += flip(a.tc[t], __popc(a.tz[t] & bd));
    acc += Acc<T>::prod(cf, psi[src]);
  }
  ((T*)a.sigma)[d] = (T)acc;
}

// ---------------------------------------------------------------- launch


static int g_support_skip = 1;  // process-wide: restrict H psi to psi's row and column support
static int g_ss_cores = 2;      // process-wide: FP64 same-spin doubles through the cores: 0 off, 1 where
                                // built, 2 where built and the FP64 state exceeds kCoreAutoBytes
static int g_mixed_mm = 2;      // process-wide: mixed pass on the matrix cores (k_mixed_m): 0 off, 1 where
                                // the row fits LDS, 2 where it fits and the state exceeds kMMAutoBytes
static int g_ss_groups = 2;     // process-wide: FP64 same-spin pass over grouped lists with this many
                                // 64-column tiles per four-wave workgroup (1, 2 or 4); 0: per-row lists

template <typename T>
static hyp_status run_mixed(Ham* Hm, HamWork* W, const void* psi, void* sigma, uint32_t* nz_b, hipStream_t st);

static int same_spin_entries(int M, int N) {
  const int s = N * (M - N);
  const int d = (N * (N - 1) / 2) * ((M - N) * (M - N - 1) / 2);
  return 1 + s + d;
}

// Build both same-spin matrices (synchronous on st).
static hyp_status build_same_spin(Ham* Hm, HamWork* W, hipStream_t st) {
  Sector* S = Hm->sec;
  W->a_nent = same_spin_entries(S->M, S->na);
  W->b_nent = same_spin_entries(S->M, S->nb);
  HYP_HIP(hipMalloc(&W->a_rank, sizeof(int) * S->da * W->a_nent));
  HYP_HIP(hipMalloc(&W->a_coef, sizeof(double) * S->da * W->a_nent));
  HYP_HIP(hipMalloc(&W->b_rank, sizeof(int) * S->db * W->b_nent));
  HYP_HIP(hipMalloc(&W->b_coef, sizeof(double) * S->db * W->b_nent));
  HYP_HIP(hipMalloc(&W->ca_rank, sizeof(int) * S->da * W->a_nent));
  HYP_HIP(hipMalloc(&W->ca_coef, sizeof(double) * S->da * W->a_nent));
  HYP_HIP(hipMalloc(&W->ca_n, sizeof(int) * S->da));
  HYP_HIP(hipMalloc(&W->cb_rank, sizeof(int) * S->db * W->b_nent));
  HYP_HIP(hipMalloc(&W->cb_coef, sizeof(double) * S->db * W->b_nent));
  HYP_HIP(hipMalloc(&W->cb_n, sizeof(int) * S->db));
  SameSpinArgs sa;
  sa.H = Hm->dev;
  sa.M = S->M;
  sa.list_rank = W->a_rank;
  sa.list_coef = W->a_coef;
  sa.nent = W->a_nent;
  sa.nrow = (int)S->da;
  sa.nel = S->na;
  sa.spin = 0;
  sa.rstr = S->d_astr;
  sa.rrank = S->d_arank;
  sa.constant = 0.0;
  HYP_LAUNCH("k_ss_build", k_ss_build, dim3((unsigned)S->da), dim3(kSSThreads), 0, st, sa);
  sa.list_rank = W->b_rank;
  sa.list_coef = W->b_coef;
  sa.nent = W->b_nent;
  sa.nrow = (int)S->db;
  sa.nel = S->nb;
  sa.spin = 1;
  sa.rstr = S->d_bstr;
  sa.rrank = S->d_brank;
  sa.constant = Hm->dev.dA;
  HYP_LAUNCH("k_ss_build", k_ss_build, dim3((unsigned)S->db), dim3(kSSThreads), 0, st, sa);
  HYP_HIP(hipGetLastError());
  HYP_HIP(hipStreamSynchronize(st));
  // grouped lists of both spins (union sources of kSSG consecutive rows)
  for (int sp = 0; sp < 2; ++sp) {
    const int nrow = (int)(sp == 0 ? S->da : S->db);
    const int nent = sp == 0 ? W->a_nent : W->b_nent;
    const int* rk = sp == 0 ? W->a_rank : W->b_rank;
    const double* cf = sp == 0 ? W->a_coef : W->b_coef;
    if (nrow > kSSGWords * 32) return HYP_OK;  // beyond the bitmap: per-row lists only
    const int ng = (nrow + kSSG - 1) / kSSG;
    int* cnt = nullptr;
    HYP_HIP(hipMalloc(&cnt, sizeof(int) * ng));
    HYP_LAUNCH("k_ssg_count", k_ssg_count, dim3((unsigned)ng), dim3(256), 0, st, rk, nent, nrow, cnt);
    std::vector<int> hc((size_t)ng);
    hipError_t e = hipMemcpyAsync(hc.data(), cnt, sizeof(int) * ng, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(cnt);
    if (e != hipSuccess) return hip_fail(e, "grouped same-spin counts");
    std::vector<int64_t> off((size_t)ng + 1, 0);
    for (int g = 0; g < ng; ++g) off[(size_t)g + 1] = off[(size_t)g] + hc[(size_t)g];
    const int64_t tot = off[(size_t)ng];
    HYP_HIP(hipMalloc(&W->g_off[sp], sizeof(int64_t) * (ng + 1)));
    HYP_HIP(hipMalloc(&W->g_rank[sp], sizeof(int) * std::max<int64_t>(1, tot)));
    HYP_HIP(hipMalloc(&W->g_coef[sp], sizeof(double) * kSSG * std::max<int64_t>(1, tot)));
    HYP_HIP(hipMalloc(&W->gc_rank[sp], sizeof(int) * std::max<int64_t>(1, tot)));
    HYP_HIP(hipMalloc(&W->gc_coef[sp], sizeof(double) * kSSG * std::max<int64_t>(1, tot)));
    HYP_HIP(hipMalloc(&W->gc_cnt[sp], sizeof(int) * ng));
    HYP_HIP(hipMemcpyAsync(W->g_off[sp], off.data(), sizeof(int64_t) * (ng + 1), hipMemcpyHostToDevice, st));
    HYP_LAUNCH("k_ssg_fill", k_ssg_fill, dim3((unsigned)ng), dim3(256), 0, st, rk, cf, nent, nrow, W->g_off[sp],
               W->g_rank[sp], W->g_coef[sp]);
    HYP_HIP(hipGetLastError());
    HYP_HIP(hipStreamSynchronize(st));
    W->g_n[sp] = ng;
  }
  W->g_ok = true;
  return HYP_OK;
}

// Tables of the core path of the same-spin doubles (both spins) and the Y
// band buffer: the slot table and core masks of each string space, each
// row's C(N, 2) Y offsets (its cores in a fixed order: pairs a < b of its
// occupied orbitals, b ascending, then a), nonzero-core flags, and the band
// width, chosen so that one band of Y (ncore * S rows) takes at most
// kCoreYBytes or an eighth of the device memory, whichever is smaller (two
// bands at 32 qubits: 51 ms per product against 55 with nine 4 GiB bands).
// Not built (the grouped lists serve) where a core has more than 48 slots.
constexpr size_t kCoreYBytes = size_t(20) << 30;
// Automatic choice: the core path where the FP64 state vector exceeds the
// 256 MiB Infinity Cache.  Below that the gathered sources stay cached and
// the grouped lists are faster than writing and reading the per-core
// products (measured: 10.3 against 11.2 ms at 28 qubits, 0.73 against 0.77
// at 24; 255 against 235 ms at 32 qubits).
constexpr size_t kCoreAutoBytes = size_t(256) << 20;

// Tables of the mixed pass on the matrix cores, where its output row fits
// LDS (M <= 16).
static hyp_status build_mixed_mm(Ham* Hm, HamWork* W, hipStream_t st) {
  Sector* S = Hm->sec;
  const int da = (int)S->da;
  if (S->M > kMaxOrb || da <= 0 || S->db <= 0 || (size_t)da * 8 + sizeof(MixedMMLds<double>) > kMMLdsMax) return HYP_OK;
  const int qr = (da + kMMCols - 1) / kMMCols * kMMSeg;  // columns per region
  const int nce = qr / kMMSeg * 16;                       // (chunk, orbital) pairs
  HYP_HIP(hipMalloc(&W->m_ent, (size_t)nce * kMMTiles * 16 * sizeof(uint32_t)));
  HYP_HIP(hipMalloc(&W->m_code, (size_t)nce * kMMTiles * 64 * sizeof(uint64_t)));
  HYP_HIP(hipMalloc(&W->m_nt, (size_t)nce));
  HYP_HIP(hipMalloc(&W->m_sel, sizeof(int)));
  HYP_LAUNCH("k_mm_tables", k_mm_tables, dim3((unsigned)nce), dim3(64), 0, st, S->M, da, qr, S->d_astr, S->d_arank,
             Hm->dev.abJa, Hm->dev.sJ, W->m_ent, W->m_code, W->m_nt);
  HYP_HIP(hipGetLastError());
  W->m_qr = qr;
  W->m_ok = true;
  return HYP_OK;
}

static hyp_status build_core_path(Ham* Hm, HamWork* W, hipStream_t st) {
  Sector* S = Hm->sec;
  size_t ycap = kCoreYBytes;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    HYP_HIP(hipGetDevice(&dev));
    HYP_HIP(hipGetDeviceProperties(&prop, dev));
    ycap = std::min(ycap, (size_t)prop.totalGlobalMem / 8);
  }
  for (int sp = 0; sp < 2; ++sp) {
    const int N = sp == 0 ? S->na : S->nb;
    if (N >= 2 && S->M - N >= 2 && core_space(S->M, N).S > 48) return HYP_OK;
  }
  size_t ybytes = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int N = sp == 0 ? S->na : S->nb;
    const int nrow = (int)(sp == 0 ? S->da : S->db), ncol = (int)(sp == 0 ? S->db : S->da);
    const RankTables& R = sp == 0 ? S->h_arank : S->h_brank;
    const std::vector<uint32_t>& str = sp == 0 ? S->h_astr : S->h_bstr;
    W->k_nuse[sp] = 1 + N * (S->M - N);
    const CoreSpace cs = core_space(S->M, N);
    W->k_band[sp] = ncol;
    HYP_HIP(hipMalloc(&W->k_rowany[sp], (size_t)std::max(1, nrow) * sizeof(int)));
    if (cs.ncore == 0) continue;  // no same-spin double
    std::vector<int> rows;
    std::vector<uint32_t> masks;
    hyp_status r = core_tables_host(S->M, N, R, rows, masks);
    if (r != HYP_OK) return r;
    const int npair = N * (N - 1) / 2;
    std::vector<int> yoff((size_t)nrow * npair);
    // colex rank of an (N - 2)-subset: sum over its sorted orbitals o_t of C(o_t, t + 1)
    auto binom = [](int n, int k) -> int64_t {
      if (k < 0 || n < k) return 0;
      int64_t v = 1;
      for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
      return v;
    };
    for (int row = 0; row < nrow; ++row) {
      const uint32_t sv = str[(size_t)row];
      int occ[16], no = 0;
      for (int o = 0; o < S->M; ++o)
        if (sv >> o & 1u) occ[no++] = o;
      int m = 0;
      for (int bi = 1; bi < no; ++bi)
        for (int ai = 0; ai < bi; ++ai) {
          const int oa = occ[ai], ob = occ[bi];
          const uint32_t K = sv & ~(1u << oa) & ~(1u << ob);
          int64_t crank = 0;
          int t = 0;
          for (int o = 0; o < S->M; ++o)
            if (K >> o & 1u) crank += binom(o, ++t);
          int u = -1, wv = -1, c = 0;
          for (int o = 0; o < S->M; ++o)
            if (!(K >> o & 1u)) {
              if (o == oa) u = c;
              if (o == ob) wv = c;
              ++c;
            }
          yoff[(size_t)row * npair + m++] = (int)(crank * cs.S + wv * (wv - 1) / 2 + u);
        }
    }
    W->k_ncore[sp] = (int)cs.ncore;
    W->k_S[sp] = cs.S;
    W->k_npair[sp] = npair;
    HYP_HIP(hipMalloc(&W->k_rows[sp], rows.size() * sizeof(int)));
    HYP_HIP(hipMalloc(&W->k_mask[sp], masks.size() * sizeof(uint32_t)));
    HYP_HIP(hipMalloc(&W->k_yoff[sp], yoff.size() * sizeof(int)));
    HYP_HIP(hipMalloc(&W->k_cnz[sp], (size_t)cs.ncore * sizeof(int)));
    HYP_HIP(hipMemcpy(W->k_rows[sp], rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice));
    HYP_HIP(hipMemcpy(W->k_mask[sp], masks.data(), masks.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HYP_HIP(hipMemcpy(W->k_yoff[sp], yoff.data(), yoff.size() * sizeof(int), hipMemcpyHostToDevice));
    // bands: multiples of 64 columns, one band of Y within kCoreYBytes
    const size_t yrow = (size_t)cs.ncore * cs.S * sizeof(double);
    const int64_t maxc = std::max<int64_t>(64, (int64_t)(ycap / yrow) / 64 * 64);
    const int nband = (int)((ncol + maxc - 1) / maxc);
    const int bw = (int)(((ncol + nband - 1) / nband + 63) / 64 * 64);
    W->k_band[sp] = bw;
    ybytes = std::max(ybytes, yrow * (size_t)bw);
  }
  (void)st;
  if (ybytes > 0) HYP_HIP(hipMalloc(&W->k_Y, ybytes));
  HYP_HIP(hipMalloc(&W->k_sel, 2 * sizeof(int)));
  W->k_ok = true;
  return HYP_OK;
}

// threads per mixed-kernel workgroup: one per alpha column, at most 1024 (a
// 16-wave workgroup leaves 128 registers per lane; the kernel needs about
// 105).  FP32 rows take half the LDS, so two 512-wide workgroups fit on a CU
// and one's row staging overlaps the other's products.
static int pick_threads(int da, hyp_dtype dt) {
  return std::max(64, std::min(dt == HYP_F32 ? 512 : 1024, (da + 63) / 64 * 64));
}

template <typename T>
static hyp_status run_structured(Ham* Hm, HamWork* W, const void* psi, void* sigma,
                                 hipStream_t st) {
  Sector* S = Hm->sec;
  const int da = (int)S->da, db = (int)S->db;
  const bool skip = g_support_skip != 0;
  uint32_t* nz_b = skip ? W->nz : nullptr;       // beta rows of psi
  uint32_t* nz_a = skip ? W->nz + db : nullptr;  // alpha columns of psi (rows of psi^T)
  if (skip) {
    const int n = da + db;
    HYP_LAUNCH("k_clear_u32", k_clear_u32, dim3((unsigned)std::min(1024, (n + 255) / 256)), dim3(256), 0, st,
               W->nz, n);
  }
  // psi^T for the alpha-row pass, and psi's row and column support
  dim3 tg((da + 63) / 64, (db + 63) / 64);
  HYP_LAUNCH("k_transpose", k_transpose<T>, tg, dim3(256), 0, st, (const T*)psi, (T*)W->psi_t, db, da, nz_b,
             nz_a);
  if (sizeof(T) == 8 && W->k_ok && (g_ss_cores == 1 || (g_ss_cores == 2 && (size_t)S->dim * 8 > kCoreAutoBytes))) {
    // FP64: the singles and diagonal from the heads of the per-row lists,
    // the doubles through the cores, one column band at a time
    for (int sp = 0; sp < 2; ++sp) {
      const int nrow = sp == 0 ? da : db, ncol = sp == 0 ? db : da;
      const int nent = sp == 0 ? W->a_nent : W->b_nent;
      const uint32_t* flags = sp == 0 ? nz_a : nz_b;
      if (skip) {
        HYP_LAUNCH("k_ss_compact", k_ss_compact, dim3((unsigned)((nrow + 3) / 4)), dim3(256), 0, st,
                   sp == 0 ? W->a_rank : W->b_rank, sp == 0 ? W->a_coef : W->b_coef, nent, W->k_nuse[sp], nrow,
                   flags, sp == 0 ? W->ca_rank : W->cb_rank, sp == 0 ? W->ca_coef : W->cb_coef,
                   sp == 0 ? W->ca_n : W->cb_n);
        if (W->k_ncore[sp] > 0)
          HYP_LAUNCH("k_core_flags", k_core_flags, dim3((unsigned)((W->k_ncore[sp] + 255) / 256)), dim3(256), 0, st,
                     W->k_rows[sp], W->k_ncore[sp], W->k_S[sp], flags, W->k_cnz[sp]);
        HYP_LAUNCH("k_row_any", k_row_any, dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0, st, W->k_yoff[sp],
                   W->k_npair[sp], std::max(1, W->k_S[sp]), W->k_cnz[sp], sp == 0 ? W->ca_n : W->cb_n, nrow,
                   W->k_rowany[sp]);
        if (W->g_ok) {
          // a sparse support takes the grouped lists (selected on the device)
          HYP_LAUNCH("k_ss_select", k_ss_select, dim3(1), dim3(1024), 0, st, flags, nrow, W->k_sel + sp);
          HYP_LAUNCH("k_ssg_compact", k_ssg_compact, dim3((unsigned)((W->g_n[sp] + 3) / 4)), dim3(256), 0, st,
                     W->g_off[sp], W->g_rank[sp], W->g_coef[sp], W->g_n[sp], flags, W->gc_rank[sp], W->gc_coef[sp],
                     W->gc_cnt[sp], (const int*)(W->k_sel + sp));
        }
      }
      const int* sel = (skip && W->g_ok) ? W->k_sel + sp : nullptr;
      const void* in = sp == 0 ? (const void*)W->psi_t : psi;
      SSApplyArgs sa{};
      sa.in = in;
      sa.out = sp == 0 ? W->part_a : W->part_b;
      sa.list_rank = skip ? (sp == 0 ? W->ca_rank : W->cb_rank) : (sp == 0 ? W->a_rank : W->b_rank);
      sa.list_coef = skip ? (sp == 0 ? W->ca_coef : W->cb_coef) : (sp == 0 ? W->a_coef : W->b_coef);
      sa.list_n = skip ? (sp == 0 ? W->ca_n : W->cb_n) : nullptr;
      sa.nent = nent;
      sa.nuse = W->k_nuse[sp];
      sa.nrow = nrow;
      sa.ncol = ncol;
      sa.nrb = (nrow + 3) / 4;
      sa.Y = W->k_Y;
      sa.ldy = W->k_band[sp];
      sa.yoff = W->k_yoff[sp];
      sa.npair = W->k_npair[sp];
      sa.S = std::max(1, W->k_S[sp]);
      sa.cnz = skip ? W->k_cnz[sp] : nullptr;
      sa.row_any = skip ? W->k_rowany[sp] : nullptr;
      sa.sel = sel;
      SSCoreArgs ca{};
      ca.in = (const double*)in;
      ca.ld = ncol;
      ca.rows = W->k_rows[sp];
      ca.masks = W->k_mask[sp];
      ca.ncore = W->k_ncore[sp];
      ca.S = W->k_S[sp];
      ca.M = S->M;
      ca.spin = sp;
      ca.per_xcd = (ca.ncore + 7) / 8;
      ca.wJ = Hm->dev.wJ;
      ca.wF = Hm->dev.wF;
      ca.Y = W->k_Y;
      ca.ldy = W->k_band[sp];
      ca.cnz = skip ? W->k_cnz[sp] : nullptr;
      ca.sel = sel;
      const int bw = W->k_band[sp];
      for (int c0 = 0; c0 < ncol; c0 += bw) {
        const int nc = std::min(bw, ncol - c0);
        if (ca.ncore > 0) {
          ca.c0 = c0;
          ca.nc = nc;
          ca.dma = (((uintptr_t)in & 15u) == 0 && ncol % 2 == 0 && c0 % 2 == 0) ? 1 : 0;
          HYP_HIP(hipFuncSetAttribute((const void*)k_ss_core, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(2 * kCoreBuf)));
          HYP_LAUNCH("k_ss_core", k_ss_core, dim3((unsigned)(8 * ca.per_xcd)), dim3(256), 2 * kCoreBuf, st, ca);
        }
        sa.c0 = c0;
        sa.nc = nc;
        sa.ntiles = (nc + 63) / 64;
        const int64_t nblk = (int64_t)8 * ((sa.ntiles + 7) / 8) * sa.nrb;
        HYP_LAUNCH("k_ss_apply", (k_ss_apply<T, true>), dim3((unsigned)nblk), dim3(256), 0, st, sa);
      }
      if (sel) {
        SSGArgs ga;
        ga.in = in;
        ga.out = sp == 0 ? W->part_a : W->part_b;
        ga.off = W->g_off[sp];
        ga.urank = W->gc_rank[sp];
        ga.ucoef = W->gc_coef[sp];
        ga.cnt = W->gc_cnt[sp];
        ga.nrow = nrow;
        ga.ncol = ncol;
        ga.ngroups = W->g_n[sp];
        ga.sel = sel;
        ga.ntq = (ncol + 127) / 128;
        const int64_t nblk = (int64_t)8 * ((ga.ntq + 7) / 8) * ((ga.ngroups + 1) / 2);
        HYP_LAUNCH("k_ss_apply_sparse", (k_ss_apply_g<T, 2>), dim3((unsigned)nblk), dim3(256), 0, st, ga);
      }
    }
    return run_mixed<T>(Hm, W, psi, sigma, nz_b, st);
  }
  if (sizeof(T) == 8 && g_ss_groups != 0 && W->g_ok) {
    // FP64: grouped lists (support-restricted copies when skipping); FP32
    // storage keeps the per-row lists (measured: 35 against 29 ms at 32 qubits)
    for (int sp = 0; sp < 2; ++sp) {
      const int ng = W->g_n[sp];
      if (skip)
        HYP_LAUNCH("k_ssg_compact", k_ssg_compact, dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, st, W->g_off[sp],
                   W->g_rank[sp], W->g_coef[sp], ng, sp == 0 ? nz_a : nz_b, W->gc_rank[sp], W->gc_coef[sp],
                   W->gc_cnt[sp], (const int*)nullptr);
      SSGArgs ga;
      ga.in = sp == 0 ? (const void*)W->psi_t : psi;
      ga.out = sp == 0 ? W->part_a : W->part_b;
      ga.off = W->g_off[sp];
      ga.urank = skip ? W->gc_rank[sp] : W->g_rank[sp];
      ga.ucoef = skip ? W->gc_coef[sp] : W->g_coef[sp];
      ga.cnt = skip ? W->gc_cnt[sp] : nullptr;
      ga.nrow = sp == 0 ? da : db;
      ga.ncol = sp == 0 ? db : da;
      ga.ngroups = ng;
      ga.sel = nullptr;
      const int kw = g_ss_groups;  // tiles per workgroup: 1, 2 or 4
      ga.ntq = (ga.ncol + 64 * kw - 1) / (64 * kw);
      const int ngq = (ng + 4 / kw - 1) / (4 / kw);
      const int64_t nblk = (int64_t)8 * ((ga.ntq + 7) / 8) * ngq;
      if (kw == 4)
        HYP_LAUNCH("k_ss_apply", (k_ss_apply_g<T, 4>), dim3((unsigned)nblk), dim3(256), 0, st, ga);
      else if (kw == 2)
        HYP_LAUNCH("k_ss_apply", (k_ss_apply_g<T, 2>), dim3((unsigned)nblk), dim3(256), 0, st, ga);
      else
        HYP_LAUNCH("k_ss_apply", (k_ss_apply_g<T, 1>), dim3((unsigned)nblk), dim3(256), 0, st, ga);
    }
    return run_mixed<T>(Hm, W, psi, sigma, nz_b, st);
  }
  if (skip) {
    // same-spin matrices restricted to source rows in the support
    HYP_LAUNCH("k_ss_compact", k_ss_compact, dim3((unsigned)((da + 3) / 4)), dim3(256), 0, st, W->a_rank,
               W->a_coef, W->a_nent, W->a_nent, da, nz_a, W->ca_rank, W->ca_coef, W->ca_n);
    HYP_LAUNCH("k_ss_compact", k_ss_compact, dim3((unsigned)((db + 3) / 4)), dim3(256), 0, st, W->b_rank,
               W->b_coef, W->b_nent, W->b_nent, db, nz_b, W->cb_rank, W->cb_coef, W->cb_n);
  }
  // alpha rows (over psi^T): rows = alpha strings, columns = beta strings
  SSApplyArgs sa{};
  sa.in = W->psi_t;
  sa.out = W->part_a;
  sa.list_rank = skip ? W->ca_rank : W->a_rank;
  sa.list_coef = skip ? W->ca_coef : W->a_coef;
  sa.list_n = skip ? W->ca_n : nullptr;
  sa.nent = W->a_nent;
  sa.nuse = W->a_nent;
  sa.nrow = da;
  sa.ncol = db;
  sa.c0 = 0;
  sa.nc = db;
  sa.ntiles = (db + 63) / 64;
  sa.nrb = (da + 3) / 4;
  int64_t nb_a = (int64_t)8 * ((sa.ntiles + 7) / 8) * sa.nrb;
  HYP_LAUNCH("k_ss_apply", (k_ss_apply<T, false>), dim3((unsigned)nb_a), dim3(256), 0, st, sa);
  // beta rows (over psi), the constant (identity) term folded into their diagonal
  sa.in = psi;
  sa.out = W->part_b;
  sa.list_rank = skip ? W->cb_rank : W->b_rank;
  sa.list_coef = skip ? W->cb_coef : W->b_coef;
  sa.list_n = skip ? W->cb_n : nullptr;
  sa.nent = W->b_nent;
  sa.nuse = W->b_nent;
  sa.nrow = db;
  sa.ncol = da;
  sa.c0 = 0;
  sa.nc = da;
  sa.ntiles = (da + 63) / 64;
  sa.nrb = (db + 3) / 4;
  int64_t nb_b = (int64_t)8 * ((sa.ntiles + 7) / 8) * sa.nrb;
  HYP_LAUNCH("k_ss_apply", (k_ss_apply<T, false>), dim3((unsigned)nb_b), dim3(256), 0, st, sa);
  return run_mixed<T>(Hm, W, psi, sigma, nz_b, st);
}

// The mixed pass (adds the two same-spin partials).
// The matrix-core form serves this Hamiltonian and storage size.
static bool mixed_mm_applies(const Sector* S, const HamWork* W, size_t tsize) {
  const size_t lds = (size_t)S->da * 8 + (tsize == 8 ? sizeof(MixedMMLds<double>) : sizeof(MixedMMLds<float>));
  return g_mixed_mm != 0 && W->m_ok && lds <= kMMLdsMax &&
         (g_mixed_mm == 1 || (size_t)S->dim * 8 > kMMAutoBytes);
}

template <typename T>
static hyp_status run_mixed(Ham* Hm, HamWork* W, const void* psi, void* sigma, uint32_t* nz_b, hipStream_t st) {
  Sector* S = Hm->sec;
  const int da = (int)S->da, db = (int)S->db;
  MixedArgs ma;
  ma.psi = psi;
  ma.pa_t = W->part_a;
  ma.pb = W->part_b;
  ma.sigma = sigma;
  ma.M = S->M;
  ma.na = S->na;
  ma.nb = S->nb;
  ma.da = da;
  ma.db = db;
  ma.astr = S->d_astr;
  ma.bstr = S->d_bstr;
  ma.arank = S->d_arank;
  ma.brank = S->d_brank;
  ma.H = Hm->dev;
  ma.row_nz = nz_b;
  ma.sel = nullptr;
  const int nt = Hm->threads[sizeof(T) == 4 ? 1 : 0];
  ma.nchunk = (da + nt - 1) / nt;
  const size_t mshm = (size_t)da * 8;  // the output row in FP64
  if (mixed_mm_applies(S, W, sizeof(T))) {
    // under support skipping a sparse support takes the vector forms, whose
    // work follows the kept stages (chosen on the device; both launched)
    if (nz_b) {
      HYP_LAUNCH("k_ss_select", k_ss_select, dim3(1), dim3(1024), 0, st, nz_b, db, W->m_sel);
      ma.sel = W->m_sel;
    }
    const bool vec = ((uintptr_t)psi & 15u) == 0 && ((size_t)da * sizeof(T)) % 16 == 0;
    const void* kf = vec ? (const void*)k_mixed_m<T, 1> : (const void*)k_mixed_m<T, 0>;
    HYP_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mshm));
    if (vec)
      HYP_LAUNCH("k_mixed_m", (k_mixed_m<T, 1>), dim3((unsigned)db), dim3(1024), mshm, st, ma, W->m_ent, W->m_code,
                 W->m_nt, W->m_qr, W->m_qr / kMMSeg);
    else
      HYP_LAUNCH("k_mixed_m", (k_mixed_m<T, 0>), dim3((unsigned)db), dim3(1024), mshm, st, ma, W->m_ent, W->m_code,
                 W->m_nt, W->m_qr, W->m_qr / kMMSeg);
    HYP_HIP(hipGetLastError());
    if (!ma.sel) return HYP_OK;
  }
  if (sizeof(T) == 8 && nt == kCMixedThreads && row_staging_compact() && W->c_ok && (da % 2) == 0 &&
      ((uintptr_t)psi & 15u) == 0) {
    // compact, double-buffered staging (buffer 0 | buffer 1 at kCBuf1, each
    // with its zero slot)
    const size_t cshm = (size_t)kCBuf1 + ((size_t)W->c_max + 1) * 16;
    HYP_HIP(hipFuncSetAttribute((const void*)k_mixed_c, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cshm));
    const int64_t nblk = (int64_t)8 * ((db + 7) / 8) * ma.nchunk;
    HYP_LAUNCH("k_mixed", k_mixed_c, dim3((unsigned)nblk), dim3(nt), cshm, st, ma, W->c_bpos, W->c_blist, W->c_nb,
               (da + 1) / 2);
    HYP_HIP(hipGetLastError());
    return HYP_OK;
  }
  // the row plus one zero slot (index da) that padded excitation entries read
  const size_t shm = ((size_t)(da + 1) * sizeof(T) + 15) & ~(size_t)15;
  if (shm > 48 * 1024)
    HYP_HIP(hipFuncSetAttribute((const void*)k_mixed<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  const int64_t nblk = (int64_t)8 * ((db + 7) / 8) * ma.nchunk;
  HYP_LAUNCH("k_mixed", k_mixed<T>, dim3((unsigned)nblk), dim3(nt), shm, st, ma);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

template <typename T>
static hyp_status run_generic(Ham* Hm, const void* psi, void* sigma, hipStream_t st) {
  Sector* S = Hm->sec;
  GenericArgs g;
  g.psi = psi;
  g.sigma = sigma;
  g.M = S->M;
  g.na = S->na;
  g.nb = S->nb;
  g.da = (int)S->da;
  g.dim = S->dim;
  g.astr = S->d_astr;
  g.bstr = S->d_bstr;
  g.arank = S->d_arank;
  g.brank = S->d_brank;
  g.ngroup = Hm->n_groups;
  g.gx = Hm->d_gx;
  g.goff = Hm->d_goff;
  g.tz = Hm->d_tz;
  g.tc = Hm->d_tc;
  int64_t blocks = (S->dim + 255) / 256;
  HYP_LAUNCH("k_generic", k_generic<T>, dim3((unsigned)blocks), dim3(256), 0, st, g);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

}  // namespace hyp

using namespace hyp;

struct hyp_ham_s {
  Ham h;
  HamWork w;
};

namespace {

struct TermIn {
  uint32_t x, z;
  double c;
};

inline int popc(uint32_t v) { return __builtin_popcount(v); }

// Fold the X-groups into the structured tables.  Returns false if some group
// does not have the two-body closed form (then the generic kernel is used).
bool fold_structured(int M, const std::vector<TermIn>& t, const std::vector<int64_t>& goff,
                     std::vector<double>& dB, std::vector<double>& dC, double& dA,
                     std::vector<uint32_t>& sJ, std::vector<double>& sA, std::vector<double>& sB,
                     std::vector<uint32_t>& wJ, std::vector<double>& wF,
                     std::vector<uint32_t>& abJa, std::vector<uint32_t>& abJb,
                     std::vector<double>& abF, std::string& why) {
  const int n = 2 * M;
  const uint32_t amask = (1u << M) - 1u;
  const uint32_t bmask_q = amask << M;
  dA = 0.0;
  dB.assign(32, 0.0);
  dC.assign(32 * 32, 0.0);
  sJ.assign(2 * kMaxPairs, 0u);
  sA.assign(2 * kMaxPairs * 2, 0.0);
  sB.assign(2 * kMaxPairs * 2 * 32, 0.0);
  wJ.assign(2 * kMaxQuads, 0u);
  wF.assign((size_t)2 * kMaxQuads * 16, 0.0);
  abJa.assign(kMaxPairs, 0u);
  abJb.assign(kMaxPairs, 0u);
  abF.assign((size_t)kMaxPairs * kMaxPairs * 4, 0.0);
  std::vector<char> haveA(kMaxPairs, 0), haveB(kMaxPairs, 0);
  const size_t G = goff.size() - 1;
  for (size_t g = 0; g < G; ++g) {
    const uint32_t x = t[goff[g]].x;
    const uint32_t xa = x & amask, xb = (x >> M) & amask;
    const int ka = popc(xa), kb = popc(xb);
    if (ka == 0 && kb == 0) {
      for (int64_t i = goff[g]; i < goff[g + 1]; ++i) {
        const uint32_t z = t[i].z;
        const double c = t[i].c;
        const int w = popc(z);
        if (w > 2) {
          why = "diagonal term with more than two Z";
          return false;
        }
        // (-1)^{n_k} = 1 - 2 n_k ; (-1)^{n_k + n_l} = 1 - 2n_k - 2n_l + 4 n_k n_l
        dA += c;
        if (w >= 1) {
          int k = __builtin_ctz(z);
          dB[k] -= 2.0 * c;
          if (w == 2) {
            int l = 31 - __builtin_clz(z);
            dB[l] -= 2.0 * c;
            dC[k * 32 + l] += 4.0 * c;
          }
        }
      }
    } else if ((ka == 2 && kb == 0) || (ka == 0 && kb == 2)) {
      const int spin = ka ? 0 : 1;
      const uint32_t xs = ka ? xa : xb;
      const int p = __builtin_ctz(xs), q = 31 - __builtin_clz(xs);
      const int pid = pair_id(p, q);
      const uint32_t spin_q = spin ? bmask_q : amask;
      // find J with every z_out in {J} or {J xor e_k}
      const uint32_t z0 = t[goff[g]].z & ~x;
      uint32_t J = 0;
      bool found = false;
      for (int cand = -1; cand < n && !found; ++cand) {
        uint32_t Jc = cand < 0 ? z0 : (z0 ^ (1u << cand));
        if (Jc & x) continue;
        bool ok = true;
        for (int64_t i = goff[g]; i < goff[g + 1] && ok; ++i)
          if (popc((t[i].z & ~x) ^ Jc) > 1) ok = false;
        if (ok) {
          J = Jc;
          found = true;
        }
      }
      if (!found || (J & ~spin_q)) {
        why = "single-excitation group without a number-dressed form";
        return false;
      }
      sJ[spin * kMaxPairs + pid] = J;
      for (int O = 0; O < 2; ++O) {
        const uint32_t Om = (O ? (1u << q) : (1u << p)) << (spin * M);
        double F0 = 0.0;
        double Fk[32] = {0};
        for (int64_t i = goff[g]; i < goff[g + 1]; ++i) {
          const double v = (popc(t[i].z & Om) & 1) ? -t[i].c : t[i].c;
          const uint32_t r = (t[i].z & ~x) ^ J;
          if (r == 0)
            F0 += v;
          else
            Fk[__builtin_ctz(r)] += v;
        }
        double a0 = F0;
        for (int k = 0; k < n; ++k) a0 += Fk[k];
        sA[(spin * kMaxPairs + pid) * 2 + O] = a0;
        for (int k = 0; k < n; ++k) sB[((size_t)(spin * kMaxPairs + pid) * 2 + O) * 32 + k] = -2.0 * Fk[k];
      }
    } else if ((ka == 4 && kb == 0) || (ka == 0 && kb == 4)) {
      const int spin = ka ? 0 : 1;
      const uint32_t xs = ka ? xa : xb;
      int o[4], c = 0;
      for (int k = 0; k < M; ++k)
        if (xs & (1u << k)) o[c++] = k;
      const int qid = quad_id(o[0], o[1], o[2], o[3]);
      const uint32_t zo = t[goff[g]].z & ~x;
      const uint32_t spin_q = spin ? bmask_q : amask;
      for (int64_t i = goff[g]; i < goff[g + 1]; ++i)
        if ((t[i].z & ~x) != zo) {
          why = "same-spin double group with several Z strings";
          return false;
        }
      if (zo & ~spin_q) {
        why = "same-spin double group with a Z string on the other spin";
        return false;
      }
      wJ[spin * kMaxQuads + qid] = zo;
      for (int O4 = 0; O4 < 16; ++O4) {
        if (popc(O4) != 2) continue;
        uint32_t Om = 0;
        for (int k = 0; k < 4; ++k)
          if (O4 & (1 << k)) Om |= 1u << o[k];
        Om <<= spin * M;
        double v = 0.0;
        for (int64_t i = goff[g]; i < goff[g + 1]; ++i)
          v += (popc(t[i].z & Om) & 1) ? -t[i].c : t[i].c;
        wF[((size_t)spin * kMaxQuads + qid) * 16 + O4] = v;
      }
    } else if (ka == 2 && kb == 2) {
      const int pa_lo = __builtin_ctz(xa), pa_hi = 31 - __builtin_clz(xa);
      const int pb_lo = __builtin_ctz(xb), pb_hi = 31 - __builtin_clz(xb);
      const int pa = pair_id(pa_lo, pa_hi), pb = pair_id(pb_lo, pb_hi);
      const uint32_t zo = t[goff[g]].z & ~x;
      for (int64_t i = goff[g]; i < goff[g + 1]; ++i)
        if ((t[i].z & ~x) != zo) {
          why = "alpha-beta group with several Z strings";
          return false;
        }
      const uint32_t za = zo & amask, zb = zo & bmask_q;
      if ((haveA[pa] && abJa[pa] != za) || (haveB[pb] && abJb[pb] != zb)) {
        why = "alpha-beta Z strings do not factor by spin";
        return false;
      }
      haveA[pa] = haveB[pb] = 1;
      abJa[pa] = za;
      abJb[pb] = zb;
      for (int Oa = 0; Oa < 2; ++Oa)
        for (int Ob = 0; Ob < 2; ++Ob) {
          const uint32_t Om = (Oa ? (1u << pa_hi) : (1u << pa_lo)) |
                              ((Ob ? (1u << pb_hi) : (1u << pb_lo)) << M);
          double v = 0.0;
          for (int64_t i = goff[g]; i < goff[g + 1]; ++i)
            v += (popc(t[i].z & Om) & 1) ? -t[i].c : t[i].c;
          abF[((size_t)pa * kMaxPairs + pb) * 4 + Oa * 2 + Ob] = v;
        }
    } else {
      why = "X-mask outside the two-body classes";
      return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

hyp_status hyp_build_hamiltonian(hyp_sector sh, const uint32_t* x_mask, const uint32_t* z_mask,
                                 const double* coeff, int64_t n_terms, void* stream,
                                 hyp_ham* out) {
  Sector* S = sector_of(sh);
  if (!S || !out) return fail(HYP_ERR_ARG, "hyp_build_hamiltonian: NULL sector or out");
  if (n_terms < 0) return fail(HYP_ERR_ARG, "hyp_build_hamiltonian: n_terms < 0");
  if (n_terms > 0 && (!x_mask || !z_mask || !coeff))
    return fail(HYP_ERR_ARG, "hyp_build_hamiltonian: NULL term array");
  const int M = S->M, n = 2 * M;
  const uint32_t all = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
  const uint32_t amask = (1u << M) - 1u;
  std::vector<TermIn> t;
  t.reserve((size_t)n_terms);
  for (int64_t i = 0; i < n_terms; ++i) {
    if ((x_mask[i] & ~all) || (z_mask[i] & ~all))
      return fail(HYP_ERR_ARG, "hyp_build_hamiltonian: mask bit >= 2*n_orb");
    if (!std::isfinite(coeff[i])) return fail(HYP_ERR_ARG, "hyp_build_hamiltonian: non-finite coefficient");
    if ((popc(x_mask[i] & z_mask[i]) & 1) && coeff[i] != 0.0)
      return fail(HYP_ERR_NONREAL, "hyp_build_hamiltonian: odd number of Y (imaginary coefficient)");
    t.push_back({x_mask[i], z_mask[i], coeff[i]});
  }
  std::stable_sort(t.begin(), t.end(), [](const TermIn& a, const TermIn& b) {
    return a.x != b.x ? a.x < b.x : a.z < b.z;
  });
  // merge duplicates, c' = c (-1)^{n_Y/2}, drop exact zeros and groups that
  // cannot connect two states of this sector
  std::vector<TermIn> m;
  for (size_t i = 0; i < t.size();) {
    size_t j = i;
    double c = 0.0;
    while (j < t.size() && t[j].x == t[i].x && t[j].z == t[i].z) c += t[j++].c;
    const uint32_t x = t[i].x, xa = x & amask, xb = (x >> M) & amask;
    const int ka = popc(xa), kb = popc(xb);
    bool connects = !(ka & 1) && !(kb & 1) && ka / 2 <= std::min(S->na, M - S->na) &&
                    kb / 2 <= std::min(S->nb, M - S->nb);
    if (c != 0.0 && connects) {
      if ((popc(x & t[i].z) / 2) & 1) c = -c;
      m.push_back({x, t[i].z, c});
    }
    i = j;
  }
  std::vector<int64_t> goff;
  for (size_t i = 0; i < m.size(); ++i)
    if (i == 0 || m[i].x != m[i - 1].x) goff.push_back((int64_t)i);
  goff.push_back((int64_t)m.size());
  if (m.empty()) goff.assign(1, 0);

  hyp_ham_s* hh = new (std::nothrow) hyp_ham_s();
  if (!hh) return fail(HYP_ERR_NOMEM, "hyp_build_hamiltonian: host allocation");
  Ham& H = hh->h;
  H.sec = S;
  H.n_terms = (int64_t)m.size();
  H.n_groups = (int64_t)goff.size() - 1;
  hipStream_t st = (hipStream_t)stream;

  std::vector<double> dB, dC, sA, sB, wF, abF;
  std::vector<uint32_t> sJ, wJ, abJa, abJb;
  double dA = 0.0;
  std::string why;
  H.structured = fold_structured(M, m, goff, dB, dC, dA, sJ, sA, sB, wJ, wF, abJa, abJb, abF, why);

  std::vector<uint32_t> gx(H.n_groups), tz(m.size());
  std::vector<double> tc(m.size());
  for (int64_t g = 0; g < H.n_groups; ++g) gx[g] = m[goff[g]].x;
  for (size_t i = 0; i < m.size(); ++i) {
    tz[i] = m[i].z;
    tc[i] = m[i].c;
  }
  auto cleanup_fail = [&](hipError_t e, const char* what) {
    hyp_ham_destroy(hh);
    return hip_fail(e, what);
  };
  hipError_t e = hipSuccess;
  e = hipMalloc(&H.d_gx, std::max<size_t>(1, gx.size()) * 4);
  if (e == hipSuccess) e = hipMalloc(&H.d_goff, goff.size() * 8);
  if (e == hipSuccess) e = hipMalloc(&H.d_tz, std::max<size_t>(1, tz.size()) * 4);
  if (e == hipSuccess) e = hipMalloc(&H.d_tc, std::max<size_t>(1, tc.size()) * 8);
  if (e == hipSuccess && !gx.empty()) e = hipMemcpyAsync(H.d_gx, gx.data(), gx.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(H.d_goff, goff.data(), goff.size() * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !tz.empty()) e = hipMemcpyAsync(H.d_tz, tz.data(), tz.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !tc.empty()) e = hipMemcpyAsync(H.d_tc, tc.data(), tc.size() * 8, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return cleanup_fail(e, "hyp_build_hamiltonian: generic table upload");

  if (H.structured) {
    // one blob: doubles first, then u32 tables
    size_t nd = dB.size() + dC.size() + sA.size() + sB.size() + wF.size() + abF.size();
    size_t nu = sJ.size() + wJ.size() + abJa.size() + abJb.size();
    std::vector<unsigned char> blob(nd * 8 + nu * 4);
    size_t off = 0;
    auto putd = [&](const std::vector<double>& v) {
      size_t o = off;
      std::memcpy(blob.data() + off, v.data(), v.size() * 8);
      off += v.size() * 8;
      return o;
    };
    auto putu = [&](const std::vector<uint32_t>& v) {
      size_t o = off;
      std::memcpy(blob.data() + off, v.data(), v.size() * 4);
      off += v.size() * 4;
      return o;
    };
    size_t o_dB = putd(dB), o_dC = putd(dC), o_sA = putd(sA), o_sB = putd(sB), o_wF = putd(wF),
           o_abF = putd(abF);
    size_t o_sJ = putu(sJ), o_wJ = putu(wJ), o_abJa = putu(abJa), o_abJb = putu(abJb);
    e = hipMalloc(&H.d_blob, blob.size());
    if (e == hipSuccess) e = hipMemcpyAsync(H.d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return cleanup_fail(e, "hyp_build_hamiltonian: structured table upload");
    unsigned char* b = (unsigned char*)H.d_blob;
    H.dev.dA = dA;
    H.dev.dB = (const double*)(b + o_dB);
    H.dev.dC = (const double*)(b + o_dC);
    H.dev.sA = (const double*)(b + o_sA);
    H.dev.sB = (const double*)(b + o_sB);
    H.dev.wF = (const double*)(b + o_wF);
    H.dev.abF = (const double*)(b + o_abF);
    H.dev.sJ = (const uint32_t*)(b + o_sJ);
    H.dev.wJ = (const uint32_t*)(b + o_wJ);
    H.dev.abJa = (const uint32_t*)(b + o_abJa);
    H.dev.abJb = (const uint32_t*)(b + o_abJb);
    H.threads[0] = pick_threads((int)S->da, HYP_F64);
    H.threads[1] = pick_threads((int)S->da, HYP_F32);
    // workspace: psi^T and the two same-spin partials
    e = hipMalloc(&hh->w.psi_t, (size_t)S->dim * 8);
    if (e == hipSuccess) e = hipMalloc(&hh->w.part_a, (size_t)S->dim * 8);
    if (e == hipSuccess) e = hipMalloc(&hh->w.part_b, (size_t)S->dim * 8);
    if (e == hipSuccess) e = hipMalloc(&hh->w.nz, sizeof(uint32_t) * (size_t)(S->da + S->db));
    if (e != hipSuccess) return cleanup_fail(e, "hyp_build_hamiltonian: workspace");
    hyp_status rb = build_same_spin(&H, &hh->w, st);
    if (rb == HYP_OK) rb = build_core_path(&H, &hh->w, st);
    if (rb == HYP_OK) rb = build_mixed_mm(&H, &hh->w, st);
    if (rb != HYP_OK) {
      hyp_ham_destroy(hh);
      return rb;
    }
    // compact staging tables of the FP64 mixed pass (768-column chunks);
    // where they fit, 768 threads is the default FP64 width
    if (S->da % 2 == 0 && S->da > kCMixedThreads - 64) {
      int mx = 0;
      rb = build_compact_tables(S, kCMixedThreads, &hh->w.c_bpos, &hh->w.c_blist, &hh->w.c_nb, &mx, st);
      if (rb != HYP_OK) {
        hyp_ham_destroy(hh);
        return rb;
      }
      hh->w.c_max = mx;
      hh->w.c_ok = mx <= kCMaxBlk && (mx + kCMixedThreads - 1) / kCMixedThreads <= kCPerThread;
      if (hh->w.c_ok) H.threads[0] = kCMixedThreads;
    }
  }
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup_fail(e, "hyp_build_hamiltonian: upload sync");
  if (!H.structured) set_error(std::string("generic kernel: ") + why);
  *out = hh;
  return HYP_OK;
}

hyp_status hyp_ham_destroy(hyp_ham hh) {
  if (!hh) return HYP_OK;
  Ham& H = hh->h;
  (void)hipFree(H.d_gx);
  (void)hipFree(H.d_goff);
  (void)hipFree(H.d_tz);
  (void)hipFree(H.d_tc);
  (void)hipFree(H.d_blob);
  (void)hipFree(hh->w.psi_t);
  (void)hipFree(hh->w.part_a);
  (void)hipFree(hh->w.part_b);
  (void)hipFree(hh->w.a_rank);
  (void)hipFree(hh->w.a_coef);
  (void)hipFree(hh->w.b_rank);
  (void)hipFree(hh->w.b_coef);
  (void)hipFree(hh->w.nz);
  (void)hipFree(hh->w.ca_rank);
  (void)hipFree(hh->w.ca_coef);
  (void)hipFree(hh->w.ca_n);
  (void)hipFree(hh->w.cb_rank);
  (void)hipFree(hh->w.cb_coef);
  (void)hipFree(hh->w.cb_n);
  for (int sp = 0; sp < 2; ++sp) {
    (void)hipFree(hh->w.g_off[sp]);
    (void)hipFree(hh->w.g_rank[sp]);
    (void)hipFree(hh->w.g_coef[sp]);
    (void)hipFree(hh->w.gc_rank[sp]);
    (void)hipFree(hh->w.gc_coef[sp]);
    (void)hipFree(hh->w.gc_cnt[sp]);
  }
  for (int sp = 0; sp < 2; ++sp) {
    (void)hipFree(hh->w.k_rows[sp]);
    (void)hipFree(hh->w.k_mask[sp]);
    (void)hipFree(hh->w.k_yoff[sp]);
    (void)hipFree(hh->w.k_cnz[sp]);
    (void)hipFree(hh->w.k_rowany[sp]);
  }
  (void)hipFree(hh->w.k_Y);
  (void)hipFree(hh->w.m_ent);
  (void)hipFree(hh->w.m_code);
  (void)hipFree(hh->w.m_nt);
  (void)hipFree(hh->w.m_sel);
  (void)hipFree(hh->w.k_sel);
  (void)hipFree(hh->w.c_bpos);
  (void)hipFree(hh->w.c_blist);
  (void)hipFree(hh->w.c_nb);
  delete hh;
  return HYP_OK;
}

int hyp_ham_is_structured(hyp_ham hh) { return hh ? (hh->h.structured ? 1 : 0) : -1; }

// Autotuner of the mixed pass: times every candidate workgroup width on this
// Hamiltonian (reps applications each, HIP events on `stream`), keeps the
// fastest for later hyp_apply_h calls and returns it.  sigma is overwritten.
hyp_status hyp_tune_apply_h(hyp_ham hh, hyp_dtype dtype, const void* psi, void* sigma, int reps,
                            void* stream, int* best_threads, double* best_ms) {
  if (!hh || !psi || !sigma || reps < 1 || !best_threads || !best_ms)
    return fail(HYP_ERR_ARG, "hyp_tune_apply_h: bad argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_tune_apply_h: bad dtype");
  Ham* H = &hh->h;
  if (!H->structured) {
    *best_threads = 0;
    *best_ms = 0.0;
    return HYP_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  const int da = (int)H->sec->da;
  static const int cand[] = {128, 256, 384, 512, 640, 768, 896, 1024};
  if (mixed_mm_applies(H->sec, &hh->w, dtype == HYP_F32 ? 4 : 8)) {
    // the matrix-core form (1024 threads per beta row) takes no width: time it
    hipEvent_t e0, e1;
    HYP_HIP(hipEventCreate(&e0));
    HYP_HIP(hipEventCreate(&e1));
    hyp_status r = apply_h_internal(hh, dtype, psi, sigma, st);
    if (r == HYP_OK) HYP_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps && r == HYP_OK; ++i) r = apply_h_internal(hh, dtype, psi, sigma, st);
    float ms = 0.f;
    if (r == HYP_OK) {
      HYP_HIP(hipEventRecord(e1, st));
      HYP_HIP(hipEventSynchronize(e1));
      HYP_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != HYP_OK) return r;
    *best_threads = 1024;
    *best_ms = ms / reps;
    return HYP_OK;
  }
  hipEvent_t e0, e1;
  HYP_HIP(hipEventCreate(&e0));
  HYP_HIP(hipEventCreate(&e1));
  double bms = 1e300;
  const int ti = dtype == HYP_F32 ? 1 : 0;
  int bt = H->threads[ti];
  hyp_status r = HYP_OK;
  for (int t : cand) {
    if (t > std::max(64, (da + 63) / 64 * 64) && t != cand[0]) continue;
    H->threads[ti] = std::min(t, std::max(64, (da + 63) / 64 * 64));
    r = apply_h_internal(hh, dtype, psi, sigma, st);
    if (r != HYP_OK) break;
    HYP_HIP(hipEventRecord(e0, st));
    for (int i = 0; i < reps && r == HYP_OK; ++i) r = apply_h_internal(hh, dtype, psi, sigma, st);
    HYP_HIP(hipEventRecord(e1, st));
    HYP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    HYP_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (r == HYP_OK && ms / reps < bms) {
      bms = ms / reps;
      bt = H->threads[ti];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  H->threads[ti] = bt;
  if (r != HYP_OK) return r;
  *best_threads = bt;
  *best_ms = bms;
  return HYP_OK;
}

hyp_status hyp_set_same_spin_groups(int tiles) {
  if (tiles != 0 && tiles != 1 && tiles != 2 && tiles != 4)
    return fail(HYP_ERR_ARG, "hyp_set_same_spin_groups: tiles must be 0, 1, 2 or 4");
  g_ss_groups = tiles;
  return HYP_OK;
}

hyp_status hyp_set_same_spin_cores(int mode) {
  if (mode < 0 || mode > 2) return fail(HYP_ERR_ARG, "hyp_set_same_spin_cores: mode must be 0, 1 or 2");
  g_ss_cores = mode;
  return HYP_OK;
}

hyp_status hyp_set_mixed_matrix_cores(int mode) {
  if (mode < 0 || mode > 2) return fail(HYP_ERR_ARG, "hyp_set_mixed_matrix_cores: mode must be 0, 1 or 2");
  g_mixed_mm = mode;
  return HYP_OK;
}

hyp_status hyp_set_support_skip(int on) {
  if (on != 0 && on != 1) return fail(HYP_ERR_ARG, "hyp_set_support_skip: on must be 0 or 1");
  g_support_skip = on;
  return HYP_OK;
}

hyp_status hyp_apply_h(hyp_ham hh, hyp_dtype dtype, const void* psi, void* sigma, void* stream) {
  if (!hh || !psi || !sigma) return fail(HYP_ERR_ARG, "hyp_apply_h: NULL argument");
  if (dtype != HYP_F64 && dtype != HYP_F32) return fail(HYP_ERR_ARG, "hyp_apply_h: bad dtype");
  if (psi == sigma) return fail(HYP_ERR_ARG, "hyp_apply_h: psi and sigma alias");
  return apply_h_internal(hh, dtype, psi, sigma, (hipStream_t)stream);
}

}  // extern "C"

namespace hyp {
Ham* ham_of(hyp_ham h) { return h ? &h->h : nullptr; }
HamWork* work_of(hyp_ham h) { return h ? &h->w : nullptr; }
bool support_skip() { return g_support_skip != 0; }
int mixed_mm_mode() { return g_mixed_mm; }

hyp_status apply_h_internal(hyp_ham hh, hyp_dtype dtype, const void* psi, void* sigma,
                            hipStream_t st) {
  Ham* H = &hh->h;
  if (H->structured) {
    if (dtype == HYP_F64) return run_structured<double>(H, &hh->w, psi, sigma, st);
    return run_structured<float>(H, &hh->w, psi, sigma, st);
  }
  if (dtype == HYP_F64) return run_generic<double>(H, psi, sigma, st);
  return run_generic<float>(H, psi, sigma, st);
}
}  // namespace hyp
