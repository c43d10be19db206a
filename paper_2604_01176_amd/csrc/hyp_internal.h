// Internal declarations of the gfx950 state-vector library (not part of the
// public C ABI).  Host objects, device table layouts and launch helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hyperion_mi355x.h"

namespace hyp {

constexpr int kMaxOrb = 16;           // n <= 32 qubits
constexpr int kMaxPairs = 120;        // C(16,2)
constexpr int kMaxQuads = 1820;       // C(16,4)

// Thread-local error text behind hyp_last_error().
void set_error(const std::string& msg);
hyp_status fail(hyp_status st, const std::string& msg);
hyp_status hip_fail(hipError_t e, const char* what);

// Event bracket around one launch (active only while profiling is enabled).
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();
 private:
  const char* name_;
  hipStream_t st_;
  void* a_ = nullptr;
};

#define HYP_LAUNCH(name, kernel, grid, block, shm, st, ...)              \
  do {                                                                   \
    ::hyp::ProfScope ps_(name, st);                                      \
    hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);       \
  } while (0)

#define HYP_HIP(call)                                            \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ::hyp::hip_fail(e_, #call);     \
  } while (0)

// Split colex rank: for a k-subset s of {0..M-1},
//   rank(s) = lo[s & 255] + hi[s >> 8]
// because the position of every high bit among the set bits depends only on
// how many bits the low byte holds, which is k - popc(s >> 8).
struct RankTables {
  int32_t lo[256];
  int32_t hi[256];
};

// Device-side description of a sector (passed by value to kernels).
struct SectorDev {
  int M, na, nb;
  int da, db;             // C(M,na), C(M,nb)
  int64_t dim;
  const uint32_t* astr;   // [da] alpha string of each alpha rank
  const uint32_t* bstr;   // [db]
  const RankTables* arank;  // device copies
  const RankTables* brank;
  int fsign;              // 1: fermionic excitation signs; 0: qubit excitations (every sign +1)
};

// Process-wide generator kind (hyp_set_pool_kind): 0 fermionic, 1 qubit excitations.
int pool_kind();

struct Sector {
  int M = 0, na = 0, nb = 0;
  int64_t da = 0, db = 0, dim = 0;
  std::vector<uint32_t> h_astr, h_bstr;
  RankTables h_arank{}, h_brank{};
  uint32_t* d_astr = nullptr;
  uint32_t* d_bstr = nullptr;
  RankTables* d_arank = nullptr;
  RankTables* d_brank = nullptr;
  double* d_scratch = nullptr;      // reduction partials (kScratch doubles)
  double* d_pair = nullptr;         // chunk partials of the pair kernels (grow-only)
  size_t pair_cap = 0;
  int device = 0;
  SectorDev dev() const {
    SectorDev s;
    s.M = M; s.na = na; s.nb = nb; s.da = (int)da; s.db = (int)db; s.dim = dim;
    s.astr = d_astr; s.bstr = d_bstr; s.arank = d_arank; s.brank = d_brank;
    s.fsign = pool_kind() == 0 ? 1 : 0;
    return s;
  }
};
constexpr int kScratch = 8192;
constexpr int kDotBlocks = 1024;

// ---------------------------------------------------------------------------
// X-grouped Hamiltonian, structured form.
//
// Every Pauli term (x, z, c) with even n_Y becomes, on in-sector outputs d,
// c' (-1)^{popc(z & d)} with c' = c (-1)^{n_Y/2}.  Terms are grouped by x;
// each group is folded at build time into a closed evaluation over the
// occupation pattern of d (see hamiltonian.hip).  The classes of x that can
// connect two states of one (N_a, N_b) sector under a two-body Hamiltonian:
//   diag     x = 0
//   single   2 bits of one spin       (index: spin, pair id)
//   double   4 bits of one spin       (index: spin, quad id)
//   ab       2 alpha + 2 beta bits    (index: alpha pair id, beta pair id)
// ---------------------------------------------------------------------------
struct HamDev {
  // diagonal: E(d) = dA + sum_{k in occ} dB[k] + sum_{k<l in occ} dC[k][l]
  double dA;
  const double* dB;        // [32]
  const double* dC;        // [32*32] (upper triangle used)
  // singles, per spin s and pair id p (p = q(q-1)/2 + lo, lo < q):
  //   v(d) = (-1)^{popc(sJ & d)} (sA[O] + sum_{k in occ(d), k not in x} sB[O][k])
  //   O = 1 if the upper orbital of the pair is occupied in d, else 0
  const uint32_t* sJ;      // [2][120]
  const double* sA;        // [2][120][2]
  const double* sB;        // [2][120][2][32]
  // same-spin doubles, per spin and quad id (colex rank of the 4-subset):
  //   v(d) = (-1)^{popc(wJ & d)} wF[O4], O4 = 4-bit mask of which sorted
  //   orbitals of the quad are occupied in d
  const uint32_t* wJ;      // [2][1820]
  const double* wF;        // [2][1820][16]
  // alpha-beta doubles: v(d) = (-1)^{popc(abJa[pa] & d)} (-1)^{popc(abJb[pb] & d)}
  //   abF[pa][pb][Oa*2+Ob]
  const uint32_t* abJa;    // [120]
  const uint32_t* abJb;    // [120]
  const double* abF;       // [120][120][4]
};

struct Ham {
  Sector* sec = nullptr;
  bool structured = false;
  // structured tables (one device allocation)
  void* d_blob = nullptr;
  HamDev dev{};
  // generic form: groups sorted by x
  int64_t n_terms = 0, n_groups = 0;
  uint32_t* d_gx = nullptr;        // [G] x mask
  int64_t* d_goff = nullptr;       // [G+1] term offsets
  uint32_t* d_tz = nullptr;        // [T] z mask
  double* d_tc = nullptr;          // [T] c' = c (-1)^{n_Y/2}
  // launch tuning for the structured kernel
  int threads[2] = {0, 0};  // mixed-pass workgroup width per storage type: [0] FP64, [1] FP32
};

hyp_status launch_dot(Sector* S, hyp_dtype dt, const void* a, const void* b, double* out,
                      hipStream_t st);

// Copy n elements of a global row into LDS with all of a thread's loads in
// flight before its first LDS store (kUnroll independent loads per round), so
// one staging costs about one memory latency instead of one per element.
template <typename T, int kUnroll = 72 / (int)sizeof(T)>
__device__ inline void stage_row(T* __restrict__ dst, const T* __restrict__ src, int n, int tid, int nt) {
  for (int base = tid; base < n; base += nt * kUnroll) {
    T v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int c = base + u * nt;
      v[u] = c < n ? src[c] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int c = base + u * nt;
      if (c < n) dst[c] = v[u];
    }
  }
}

// Copy nbytes of a global row into LDS with direct global->LDS loads
// (global_load_lds: lane l of a wave writes its piece at the wave's uniform
// LDS base + 16 l), 16-byte pieces when the source is 16-byte aligned and
// nbytes a multiple of 16, else 4-byte pieces.  No registers hold the data
// and every piece of the row is in flight at once.  The caller's barrier
// publishes the row (the compiler waits for these loads before it).
// Requires nt % 64 == 0 and a 16-byte aligned dst.
__device__ inline void stage_row_lds(void* dst, const void* src, int nbytes, int tid, int nt) {
  const int lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  if ((((uintptr_t)s & 15u) == 0) && (nbytes & 15) == 0) {
    const int n = nbytes >> 4;
    for (int base = w * 64; base < n; base += nw * 64) {
      const int c = base + lane;
      if (c < n)
        __builtin_amdgcn_global_load_lds((const void*)(s + (size_t)c * 16),
                                         (__attribute__((address_space(3))) void*)(d + (size_t)base * 16), 16, 0, 0);
    }
  } else {
    const int n = nbytes >> 2;
    for (int base = w * 64; base < n; base += nw * 64) {
      const int c = base + lane;
      if (c < n)
        __builtin_amdgcn_global_load_lds((const void*)(s + (size_t)c * 4),
                                         (__attribute__((address_space(3))) void*)(d + (size_t)base * 4), 4, 0, 0);
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// LDS byte address of a __shared__ object, and a load from such an address
// (the address goes straight into the ds_read, no base arithmetic per access)
__device__ inline uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}
template <typename T>
__device__ inline T lds_load(uint32_t a) {
  return *(const __attribute__((address_space(3))) T*)(uintptr_t)a;
}

// Compact staging of FP64 rows (the transition-value sweep, 512-column
// chunks, and the mixed pass, 768-column chunks): a chunk stages only the
// 16-byte blocks of a source row that its columns and their alpha single
// excitations reach, into one of two LDS buffers, the second at a fixed offset that fits the
// immediate offset of a ds_read.
constexpr int kCMaxBlk = 4094;         // staged blocks per buffer: both buffers and zero slots below 2^17 B
constexpr uint32_t kCBuf1 = 65520u;    // byte offset of the second buffer
constexpr int kCPerThread = 8;         // staged blocks per thread at 512 threads
constexpr int kCThreads = 512;         // chunk width of the sweep's compact tables
constexpr int kCMixedThreads = 768;    // chunk width of the mixed pass's compact tables
// 16 bytes per lane from global memory straight into LDS at lds_wave + 16 *
// lane.  Written as one asm statement so that the compiler does not order
// later LDS reads of the other buffer behind this copy: the caller waits for
// it (s_waitcnt vmcnt(0)) and synchronises before reading what it wrote.
// m0 (the LDS base the copy reads at issue) is saved and restored inside the
// statement, so code the compiler places around it keeps its own m0.
__device__ inline void dma16(uint32_t lds_wave, const void* src) {
  uint32_t save;
  asm volatile(
      "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %2, off\n\ts_mov_b32 m0, %0"
      : "=&s"(save)
      : "s"(lds_wave), "v"(src)
      : "memory");
}

// 4 bytes per lane, as dma16.
__device__ inline void dma4(uint32_t lds_wave, const void* src) {
  uint32_t save;
  asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %2, off\n\ts_mov_b32 m0, %0"
               : "=&s"(save)
               : "s"(lds_wave), "v"(src)
               : "memory");
}

// Stage chunk blocks blk[k] (k-th group of nt blocks) of one FP64 row.
__device__ inline void stage_blocks(uint32_t buf, const double* row, const int (&blk)[kCPerThread], int nb, int tid,
                                    int nt) {
  const int lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < kCPerThread; ++k) {
    const int base = k * nt + w * 64;  // wave-uniform
    if (base < nb) {
      const uint32_t dst = (uint32_t)__builtin_amdgcn_readfirstlane(buf + (uint32_t)base * 16u);
      if (base + lane < nb) dma16(dst, row + 2 * (int64_t)blk[k]);
    }
  }
}

// shared entry points between translation units
Sector* sector_of(hyp_sector h);
Ham* ham_of(hyp_ham h);

// Workspace and string-space matrices of a structured Hamiltonian.
struct HamWork {
  void* psi_t = nullptr;      // transposed psi, storage size of the largest dtype (8 B)
  double* part_a = nullptr;   // [da][db]
  double* part_b = nullptr;   // [db][da]
  // same-spin string-space matrices (built once per Hamiltonian)
  int* a_rank = nullptr;
  double* a_coef = nullptr;
  int a_nent = 0;
  int* b_rank = nullptr;
  double* b_coef = nullptr;
  int b_nent = 0;
  // support skipping: row flags of psi ([db] beta rows, then [da] alpha
  // columns) and the support-restricted copies of the same-spin matrices
  uint32_t* nz = nullptr;
  int* ca_rank = nullptr;
  double* ca_coef = nullptr;
  int* ca_n = nullptr;
  int* cb_rank = nullptr;
  double* cb_coef = nullptr;
  int* cb_n = nullptr;
  // grouped same-spin lists (FP64 pass): per spin [0] alpha rows, [1] beta
  // rows: group offsets, union source ranks and coefficient rows, and their
  // support-restricted copies with per-group lengths
  int g_n[2] = {0, 0};
  int64_t* g_off[2] = {nullptr, nullptr};
  int* g_rank[2] = {nullptr, nullptr};
  double* g_coef[2] = {nullptr, nullptr};
  int* gc_rank[2] = {nullptr, nullptr};
  double* gc_coef[2] = {nullptr, nullptr};
  int* gc_cnt[2] = {nullptr, nullptr};
  bool g_ok = false;
  // same-spin doubles through cores (FP64; hamiltonian.hip): per spin [0]
  // alpha rows, [1] beta rows: cores, slots per core, singles-and-diagonal
  // entries at the head of each per-row list, cores per row (C(N, 2)), the
  // slot table [ncore][S], core masks, each row's Y offsets core * S + slot
  // [nrow][npair], the nonzero-core flags of support skipping, and the band
  // width (columns per launch); Y holds one band of the per-core products
  int k_ncore[2] = {0, 0};
  int k_S[2] = {0, 0};
  int k_nuse[2] = {0, 0};
  int k_npair[2] = {0, 0};
  int* k_rows[2] = {nullptr, nullptr};
  uint32_t* k_mask[2] = {nullptr, nullptr};
  int* k_yoff[2] = {nullptr, nullptr};
  int* k_cnz[2] = {nullptr, nullptr};
  int* k_rowany[2] = {nullptr, nullptr};  // support skipping: row has a kept single or a nonzero core
  int* k_sel = nullptr;                   // support skipping, per spin: 1 core path, 0 grouped lists
  int k_band[2] = {0, 0};
  double* k_Y = nullptr;
  bool k_ok = false;
  // mixed pass on the matrix cores (row-independent tables, per chunk c,
  // alpha orbital e and 16-column tile j): m_ent[((c*16 + e)*3 + j)*16 + u]
  // the source column of slot u (chunk column | alpha string << 8),
  // m_code[((c*16 + e)*3 + j)*64 + lane] the lane's four targets (16 bits
  // each: target rank | alpha-beta sign << 14 | single-dressing sign << 15;
  // 0x3fff: none), m_nt[c*16 + e] the tile count
  uint32_t* m_ent = nullptr;
  uint64_t* m_code = nullptr;
  uint8_t* m_nt = nullptr;
  int* m_sel = nullptr;  // support skipping: 1 matrix-core form, 0 k_mixed / k_mixed_c
  int m_qr = 0;
  bool m_ok = false;
  // compact staging tables of the mixed pass (768-column chunks); c_ok when
  // every chunk fits a buffer
  uint16_t* c_bpos = nullptr;
  uint16_t* c_blist = nullptr;
  int* c_nb = nullptr;
  int c_max = 0;
  bool c_ok = false;
};
HamWork* work_of(hyp_ham h);
// Compact staging tables of a string space for nt-column chunks, into new
// allocations (caller frees): per chunk the position of every 16-byte block
// of a row in its staged list (0xffff: not staged), the list, and its
// length; *max_nb = the longest list.  Synchronous on st.
hyp_status build_compact_tables(const Sector* S, int nt, uint16_t** bpos, uint16_t** blist, int** nb, int* max_nb,
                                hipStream_t st);
// process-wide row staging switch (hyp_set_row_staging): true = compact
bool row_staging_compact();
hyp_status ensure_binom();
hyp_status validate_exc(const Sector* S, hyp_exc op);
// The same rules on the device, for lists that live in device memory:
// HYP_OK, HYP_ERR_ARG (a mask bit >= 2M, |cre| != |ann|, |cre| not in {1, 2},
// cre and ann overlap) or HYP_ERR_SECTOR (N_alpha / N_beta changed).
__host__ __device__ inline int exc_status(hyp_exc op, int M) {
  const uint32_t all = (2 * M == 32) ? 0xffffffffu : ((1u << (2 * M)) - 1u);
  const uint32_t m = (1u << M) - 1u;
  if ((op.cre | op.ann) & ~all) return HYP_ERR_ARG;
  const int nc = __builtin_popcount(op.cre), na = __builtin_popcount(op.ann);
  if (nc != na || nc < 1 || nc > 2) return HYP_ERR_ARG;
  if (op.cre & op.ann) return HYP_ERR_ARG;
  if (__builtin_popcount(op.cre & m) != __builtin_popcount(op.ann & m)) return HYP_ERR_SECTOR;
  return HYP_OK;
}
// Record of the invalid excitations a gradient kernel met: rec[0] the
// largest status, rec[1] the smallest list position (read and cleared by
// hyp_pool_check).
__device__ inline void note_bad_exc(int* rec, int status, int64_t k) {
  atomicMax(&rec[0], status);
  atomicMin(&rec[1], (int)min(k, (int64_t)0x7fffffff));
}
// This device's record (device memory), or NULL on a HIP failure.
int* bad_exc_record();
hyp_status pair_scratch(Sector* S, size_t n_doubles, double** out);
hyp_status apply_h_internal(hyp_ham h, hyp_dtype dt, const void* psi, void* sigma, hipStream_t st);
// true when hyp_pool_gradients takes the transition-value sweep for this list
bool prefer_full_sweep(const Sector* S, int64_t n_ops);
// process-wide support-skipping switch (hyp_set_support_skip)
bool support_skip();
// Process-wide switch of the alpha-beta products on the matrix cores
// (hyp_set_mixed_matrix_cores): 0 off, 1 where they fit, 2 where they fit and
// the FP64 state exceeds kMMAutoBytes (H psi) or kTMAutoBytes (the sweep).
int mixed_mm_mode();
constexpr size_t kMMAutoBytes = size_t(64) << 20;
constexpr size_t kTMAutoBytes = size_t(256) << 20;
// psi's support flags ([db] beta rows, then [da] alpha columns), device
// scratch of the sweep valid until its next use on this device
hyp_status support_flags(Sector* S, hyp_dtype dt, const void* psi, const uint32_t** flags, hipStream_t st);
hyp_status launch_pool_gradients(Sector* S, hyp_dtype dt, const hyp_exc* ops_dev, int64_t n_ops,
                                 const void* psi, const void* sig, double* grad, hipStream_t st);
hyp_status launch_rotate(Sector* S, hyp_dtype dt, hyp_exc op, double theta,
                         const double* theta_dev, void* psi, hipStream_t st);
hyp_status launch_adjoint_step(Sector* S, hyp_dtype dt, hyp_exc op, const double* theta_dev,
                               void* phi, void* lam, double* part, double* grad_out,
                               hipStream_t st);
int max_rot_chunks();
size_t tdens_bytes(const Sector* S);
hyp_status launch_tdens(Sector* S, hyp_dtype dt, const hyp_exc* ops, int64_t n_ops, const void* psi,
                        const void* sig, double* grad, hipStream_t st, bool bins);

// Core Gram blocks of a string space (M orbitals, N electrons; core_gram.hip):
// the (N-2)-electron cores in colex order, S = C(F, 2) slots each (F = M - N + 2),
// Gc[core][i][j] = sum_k sigma(slot i, k) psi(slot j, k).  ncore = 0 when the
// space has no same-spin double.
struct CoreSpace {
  int F = 0, S = 0, ntile = 0;
  int64_t ncore = 0;
};
CoreSpace core_space(int M, int N);
size_t core_gram_doubles(int M, int N);
struct CoreGramCall {
  const char* name;           // profiler name of the launch
  int M, N;                   // the string space whose pairs the blocks cover
  const RankTables* rank_host;
  bool f64;                   // storage type of psi and sigma
  const void* psi;
  const void* sig;
  int64_t rs, cs;             // storage element (string r, column k) at [r * rs + k * cs]
  int nrow, K;                // strings of the space, columns (the other spin's strings)
  const int* klist;           // support skipping (else null): psi's nonzero columns,
  const int* kcount;          //   their number (device),
  const uint32_t* rflag;      //   psi's nonzero rows (flags per string)
  double* work;               // 2 * nrow * (K rounded up to even) doubles
  double* G;                  // core_gram_doubles(M, N) doubles
};
hyp_status launch_core_gram(const CoreGramCall& g, hipStream_t st);
// Host slot table rows[core][slot] (string ranks) and core masks of (M, N).
hyp_status core_tables_host(int M, int N, const RankTables& R, std::vector<int>& rows,
                            std::vector<uint32_t>& masks);

}  // namespace hyp
