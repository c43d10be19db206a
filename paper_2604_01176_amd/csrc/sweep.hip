// Full pool-gradient sweep through transition values.
//
// Same-spin doubles use Gram entries of the two states instead:
//   G_a[I][J] = sum_beta sigma[beta][I] psi[beta][J]   (alpha strings I, J)
//   G_b[I][J] = sum_alpha sigma[I][alpha] psi[J][alpha] (beta strings)
// computed only for string pairs one same-spin double apart, grouped by their
// shared core (core_gram.hip), then
// T(tau) = sum over the generator's string pairs of s G[I][J].
//
// For an excitation tau (ordered: creates i, annihilates e, per spin)
//   T(tau) = sum_D s_tau(D) sigma[tau D] psi[D]
// and the gradient of the generator A = tau - tau^dagger is
//   g = 2 <sigma|A psi> = 2 (T(tau) - T(tau^dagger)).
// Singles and alpha-beta doubles (the 72% of all pairs at 32 qubits that
// couple different beta rows, plus the alpha singles) are computed for the
// whole pool at once, organised like the mixed H psi pass: one workgroup per
// (target beta row, 768-column chunk), one thread per target alpha column
// holding sigma[I] and its alpha single excitations in registers; for the
// row itself and each beta-single source row staged in LDS, every thread
// adds s sigma[I] psi[J] to the LDS bin of its ordered alpha excitation.
// Each workgroup writes its bins for every stage to a partial buffer (no
// atomics outside LDS); a second pass sums the partials of each transition
// value in a fixed order, and a third forms the gradients.
#include "hyp_internal.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace hyp {

constexpr int kBins = kMaxPairs * 2;     // ordered single excitations of one spin
constexpr int kStageW = kBins + 1;       // alpha bins + one beta-single bin

__constant__ int c_binom_s[17][17];

__device__ inline uint32_t betw(int p, int q) {  // orbitals strictly between p < q
  return ((1u << q) - 1u) & ~((2u << p) - 1u);
}

struct TArgs {
  const void* psi;
  const void* sig;
  int M, nb, da, db;
  const uint32_t* astr;
  const uint32_t* bstr;
  const RankTables* arank;
  const RankTables* brank;
  int nchunk, nstage;   // nstage = 1 + N_b (M - N_b)
  double* part;         // [db][nchunk][nstage][kStageW]
  int fsign;            // 1 fermionic signs, 0 qubit excitations (all +1)
};

template <typename T>
__global__ void __launch_bounds__(768) k_tdens(TArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_row = (T*)smem;
  // one private bin array per wave (no contention between waves)
  __shared__ double s_wbin[12][kBins];
  __shared__ double s_bin[kStageW];
  __shared__ double s_red[12];
  const int M = a.M;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b = blockIdx.x, xcd = b & 7, jj = b >> 3;
  const int brow = (jj / a.nchunk) * 8 + xcd;
  const int chunk = jj % a.nchunk;
  if (brow >= a.db) return;
  const uint32_t bs = a.bstr[brow];
  const int col = chunk * nt + tid;
  const bool live = col < a.da;
  const uint32_t s = live ? a.astr[col] : a.astr[0];
  const T* psi = (const T*)a.psi;
  const double sv = live ? (double)((const T*)a.sig)[(int64_t)brow * a.da + col] : 0.0;
  // packed entries: source rank (14 bits) | sign (bit 14) | bin = pair*2+O (bits 15..22)
  // Every string has the same number of single excitations, na (M - na).
  // Lane l stores its n-th excitation at slot (n + l) mod that count, so the
  // lanes of a wave, whose neighbouring strings list their excitations in
  // nearly the same order, hit different bins at any one unrolled step
  // instead of queueing on one LDS address.
  const int nsx = __popc(s) * (M - __popc(s));
  const int rot = nsx ? (tid & 63) % nsx : 0;
  uint32_t ex[64];
  int ns = 0;
  {
    uint32_t occ = s;
    while (occ) {
      const int i = __ffs(occ) - 1;
      occ &= occ - 1;
      uint32_t emp = ~s & amask;
      while (emp) {
        const int e = __ffs(emp) - 1;
        emp &= emp - 1;
        const int p = min(i, e), q = max(i, e);
        const uint32_t t2 = s ^ (1u << i) ^ (1u << e);
        const uint32_t r2 = (uint32_t)(a.arank->lo[t2 & 255u] + a.arank->hi[(t2 >> 8) & 255u]);
        const uint32_t sg = __popc(betw(p, q) & s) & (uint32_t)a.fsign;
        const uint32_t bin = (uint32_t)(q * (q - 1) / 2 + p) * 2u + (i == q ? 1u : 0u);
        const uint32_t ent = r2 | (sg << 14) | (bin << 15);
        int pos = ns + rot;
        if (pos >= nsx) pos -= nsx;
#pragma unroll
        for (int x = 0; x < 64; ++x)
          if (x == pos) ex[x] = ent;
        ++ns;
      }
    }
  }
  const int nbemp = M - a.nb;
  double* out = a.part + ((int64_t)brow * a.nchunk + chunk) * a.nstage * kStageW;
  for (int stg = 0; stg < a.nstage; ++stg) {
    // stage 0: the target row itself (alpha singles); stage 1 + jb: the
    // source row of the jb-th beta single excitation of the target row
    int src = brow;
    double sb = 1.0;
    if (stg > 0) {
      const int jb = stg - 1;
      int io = jb / nbemp, ie = jb % nbemp;
      uint32_t occ = bs, emp = ~bs & amask;
      for (int j = 0; j < io; ++j) occ &= occ - 1;
      for (int j = 0; j < ie; ++j) emp &= emp - 1;
      const int i = __ffs(occ) - 1, e = __ffs(emp) - 1;
      const uint32_t bs2 = bs ^ (1u << i) ^ (1u << e);
      src = a.brank->lo[bs2 & 255u] + a.brank->hi[(bs2 >> 8) & 255u];
      sb = (__popc(betw(min(i, e), max(i, e)) & bs) & a.fsign) ? -1.0 : 1.0;
    }
    for (int x = tid; x < 12 * kBins; x += nt) s_wbin[x / kBins][x % kBins] = 0.0;
    const T* srow = psi + (int64_t)src * a.da;
    stage_row_lds(s_row, srow, a.da * (int)sizeof(T), tid, nt);
    __syncthreads();
    const double w = sb * sv;
    if (live) {
#pragma unroll
      for (int x = 0; x < 64; ++x) {
        if (x < ns) {
          const uint32_t e2 = ex[x];
          double v;
          if (sizeof(T) == 4)
            v = (double)((float)sv * (float)s_row[e2 & 0x3fffu]) * sb;
          else
            v = w * (double)s_row[e2 & 0x3fffu];
          atomicAdd(&s_wbin[tid >> 6][(e2 >> 15) & 0xffu], (e2 >> 14) & 1u ? -v : v);
        }
      }
    }
    // beta single with the alpha identity: sigma[I] psi[J] at the same column
    double d = 0.0;
    if (stg > 0 && live) {
      if (sizeof(T) == 4)
        d = (double)((float)sv * (float)s_row[col]) * sb;
      else
        d = w * (double)s_row[col];
    }
    for (int o = 32; o > 0; o >>= 1) d += __shfl_down(d, o, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int wv = 0; wv < nt / 64; ++wv) t += s_red[wv];
      s_bin[kBins] = t;
    }
    for (int x = tid; x < kBins; x += nt) {
      double t = 0.0;
      for (int wv = 0; wv < nt / 64; ++wv) t += s_wbin[wv][x];
      s_bin[x] = t;
    }
    __syncthreads();
    for (int x = tid; x < kStageW; x += nt) out[(int64_t)stg * kStageW + x] = s_bin[x];
    __syncthreads();
  }
}

// Row-batched form of the same transition values, without atomics in the
// inner loop.  A workgroup owns one ordered beta excitation eb (or, for the
// alpha singles, a slice of rows paired with themselves) and one chunk of
// target alpha columns, and walks every (target row, source row) pair of eb:
// the source row is staged through LDS, and each thread keeps one FP64 sum per
// alpha excitation of its column in registers,
//   acc[x] += s_eb * sigma[target][J] * psi[source][I_x],
// plus the alpha-identity sum for the beta single itself.  The alpha signs and
// bins are applied once, when the sums are flushed.
struct TRArgs {
  const void* psi;
  const void* sig;
  const int* sel;     // device-side choice under support skipping: these kernels run where *sel == 0 (null: always)
  int M, da, db;
  const uint32_t* astr;
  const RankTables* arank;
  const int2* rows;   // [n_eb][K]: (source row, target row | sign << 31)
  int K, Kid;         // row pairs per beta excitation; rows per identity slice
  int nsx;            // alpha single excitations of every string, N_a (M - N_a)
  int n_eb, n_id, nchunk;
  double* part;       // [n_eb + n_id][nchunk][kStageW]
  // support skipping (null: every row): row pairs kept per beta excitation
  // (rows then holds the kept pairs first, in order), and the ordered list
  // of psi's nonzero rows with its length, split over the identity slices
  const int* rcount;
  const int* idrows;
  const int* n_idrows;
  int fsign;          // 1 fermionic signs, 0 qubit excitations (all +1)
};

// LDS byte offsets (source rank * element size) of a string's alpha single
// excitations in the staged row, in the enumeration order (occupied i
// ascending, then empty e ascending); unused slots hold pad; *ns receives
// their number.
template <typename T>
__device__ inline void alpha_sources(uint32_t s, uint32_t amask, const RankTables* R, uint32_t pad,
                                     uint32_t (&ex)[64], int* ns) {
#pragma unroll
  for (int x = 0; x < 64; ++x) ex[x] = pad;
  int n = 0;
  uint32_t occ = s;
  while (occ) {
    const int i = __ffs(occ) - 1;
    occ &= occ - 1;
    uint32_t emp = ~s & amask;
    while (emp) {
      const int e = __ffs(emp) - 1;
      emp &= emp - 1;
      const uint32_t t2 = s ^ (1u << i) ^ (1u << e);
      const uint32_t off = (uint32_t)(R->lo[t2 & 255u] + R->hi[(t2 >> 8) & 255u]) * (uint32_t)sizeof(T);
#pragma unroll
      for (int x = 0; x < 64; ++x)
        if (x == n) ex[x] = off;
      ++n;
    }
  }
  *ns = n;
}

// Bins (8 bits each, four per register) and signs (one bit each) of the same
// excitations, in the same order.
__device__ inline void alpha_bins(uint32_t s, uint32_t amask, uint32_t (&bins)[16], uint64_t* signs) {
  int n = 0;
  uint64_t sgm = 0;
  uint32_t occ = s;
  while (occ) {
    const int i = __ffs(occ) - 1;
    occ &= occ - 1;
    uint32_t emp = ~s & amask;
    while (emp) {
      const int e = __ffs(emp) - 1;
      emp &= emp - 1;
      const int p = min(i, e), q = max(i, e);
      if (__popc(betw(p, q) & s) & 1) sgm |= 1ull << n;
      const uint32_t bin = (uint32_t)(q * (q - 1) / 2 + p) * 2u + (i == q ? 1u : 0u);
#pragma unroll
      for (int x = 0; x < 16; ++x)
        if ((n >> 2) == x) bins[x] = (bins[x] & ~(0xffu << ((n & 3) * 8))) | (bin << ((n & 3) * 8));
      ++n;
    }
  }
  *signs = sgm;
}

template <typename T>
__global__ void __launch_bounds__(512) k_tdens_rows(TRArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_row = (T*)smem;
  __shared__ double s_red[8];
  if (a.sel && *a.sel != 0) return;
  const int M = a.M;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, nt = blockDim.x;
  // XCD-aware: the column chunks of one slot run on one XCD and stage the
  // same source rows at about the same time
  const int b = blockIdx.x, xcd = b & 7, jj = b >> 3;
  const int slot = (jj / a.nchunk) * 8 + xcd;
  const int chunk = jj % a.nchunk;
  if (slot >= a.n_eb + a.n_id) return;
  const int col = chunk * nt + tid;
  const bool live = col < a.da;
  const uint32_t s = live ? a.astr[col] : a.astr[0];
  // unused excitation slots read the zero slot s_row[da]
  uint32_t ex[64];
  int ns = 0;
  // absolute LDS addresses: base of the staged row plus the source offset
  const uint32_t rbase = lds_addr(s_row);
  alpha_sources<T>(s, amask, a.arank, (uint32_t)a.da * (uint32_t)sizeof(T), ex, &ns);
#pragma unroll
  for (int x = 0; x < 64; ++x) ex[x] += rbase;
  double acc[64];
#pragma unroll
  for (int x = 0; x < 64; ++x) acc[x] = 0.0;
  double acc_id = 0.0;
  const bool ident = slot >= a.n_eb;
  const int row0 = ident ? (slot - a.n_eb) * a.Kid : 0;
  int nrows;
  if (ident)
    nrows = a.idrows ? max(0, min(a.Kid, *a.n_idrows - row0)) : min(a.Kid, a.db - row0);
  else
    nrows = a.rcount ? a.rcount[slot] : a.K;
  const T* psi = (const T*)a.psi;
  const T* sig = (const T*)a.sig;
  if (tid == 0) s_row[a.da] = T(0);
  const int2* rl = a.rows + (int64_t)(ident ? 0 : slot) * a.K;
  auto pair_at = [&](int k) -> int2 {
    if (!ident) return rl[k];
    const int r = a.idrows ? a.idrows[row0 + k] : row0 + k;
    return make_int2(r, r);
  };
  // the row pair of the next iteration is read one iteration ahead, so its
  // latency is off the path to the staging loads
  int2 cur = nrows > 0 ? pair_at(0) : make_int2(0, 0);
  for (int k = 0; k < nrows; ++k) {
    const int2 nxt = (k + 1 < nrows) ? pair_at(k + 1) : cur;
    const int src = cur.x, tgt = cur.y & 0x7fffffff;
    const double sb = cur.y < 0 ? -1.0 : 1.0;
    __syncthreads();
    const T sv = live ? sig[(int64_t)tgt * a.da + col] : T(0);
    stage_row_lds(s_row, psi + (int64_t)src * a.da, a.da * (int)sizeof(T), tid, nt);
    __syncthreads();
    cur = nxt;
    if (live) {
      // groups of eight slots, each behind one uniform guard (nsx is a
      // kernel argument; slots past a string's excitations read the zero
      // slot): a group is one basic block with eight LDS reads in flight,
      // then their eight products
      const double w = sb * (double)sv;
#pragma unroll
      for (int g8 = 0; g8 < 8; ++g8) {
        if (g8 * 8 < a.nsx) {
          T v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = lds_load<T>(ex[g8 * 8 + j]);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (sizeof(T) == 4)
              acc[g8 * 8 + j] += (double)((float)sv * (float)v[j]) * sb;
            else
              acc[g8 * 8 + j] += w * (double)v[j];
          }
        }
      }
      if (!ident) {
        if (sizeof(T) == 4)
          acc_id += (double)((float)sv * (float)s_row[col]) * sb;
        else
          acc_id += w * (double)s_row[col];
      }
    }
  }
  // flush: per-wave LDS bins (the row buffer is free now), then one slot of
  // the partial buffer per (slot, chunk)
  __syncthreads();
  double* s_bins = (double*)smem;  // [nt / 64][kBins]
  const int nw = nt >> 6;
  for (int i = tid; i < nw * kBins; i += nt) s_bins[i] = 0.0;
  __syncthreads();
  if (live) {
    uint32_t bins[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) bins[x] = 0u;
    uint64_t signs = 0;
    alpha_bins(s, amask, bins, &signs);
    if (!a.fsign) signs = 0;
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      if (x < ns) {
        const uint32_t bin = (bins[x >> 2] >> ((x & 3) * 8)) & 0xffu;
        atomicAdd(&s_bins[(tid >> 6) * kBins + bin], ((signs >> x) & 1ull) ? -acc[x] : acc[x]);
      }
    }
  }
  double d = acc_id;
  for (int o = 32; o > 0; o >>= 1) d += __shfl_down(d, o, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = d;
  __syncthreads();
  double* out = a.part + ((int64_t)slot * a.nchunk + chunk) * kStageW;
  for (int x = tid; x < kBins; x += nt) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_bins[w * kBins + x];
    out[x] = t;
  }
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_red[w];
    out[kBins] = t;
  }
}

// ---------------------------------------------------------------- compact staging
// A workgroup of the row-batched kernel reads, from each staged source row,
// only the amplitudes its own columns' alpha singles reach, plus its own
// columns.  Over a chunk of consecutive colex ranks these cluster: for
// 512-column chunks of the 16-orbital, 8-electron string space they are 43%
// of the row on average (52% at most), in the same proportion of 16-byte
// blocks.  k_tdens_rows_c stages just those blocks (FP64 rows), which leaves
// room for two buffers: the copy of the next row pair runs while this one's
// products are formed.  Per-chunk tables, built once per string space:
//   bpos[c][b]  position of 16-byte block b in chunk c's staged list
//   blist[c][i] the staged blocks in ascending order, nblk_c[c] of them.
__global__ void k_cs_mark(int da, int nt, int M, const uint32_t* __restrict__ astr, const RankTables* __restrict__ R,
                          int nblk, uint8_t* __restrict__ mark) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= da) return;
  uint8_t* m = mark + (int64_t)(col / nt) * nblk;
  const uint32_t s = astr[col], amask = (1u << M) - 1u;
  m[col >> 1] = 1;
  uint32_t occ = s;
  while (occ) {
    const int i = __ffs(occ) - 1;
    occ &= occ - 1;
    uint32_t emp = ~s & amask;
    while (emp) {
      const int e = __ffs(emp) - 1;
      emp &= emp - 1;
      const uint32_t t2 = s ^ (1u << i) ^ (1u << e);
      m[(R->lo[t2 & 255u] + R->hi[(t2 >> 8) & 255u]) >> 1] = 1;
    }
  }
}

// One workgroup per chunk: positions of the marked blocks, in block order.
__global__ void __launch_bounds__(256) k_cs_scan(const uint8_t* __restrict__ mark, int nblk,
                                                 uint16_t* __restrict__ bpos, uint16_t* __restrict__ blist,
                                                 int* __restrict__ nblk_c) {
  __shared__ int s_cnt[256];
  const int c = blockIdx.x, t = threadIdx.x;
  const uint8_t* m = mark + (int64_t)c * nblk;
  const int per = (nblk + 255) / 256;
  const int b0 = min(nblk, t * per), b1 = min(nblk, b0 + per);
  int n = 0;
  for (int b = b0; b < b1; ++b) n += m[b] ? 1 : 0;
  s_cnt[t] = n;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < 256; ++i) {
      const int v = s_cnt[i];
      s_cnt[i] = run;
      run += v;
    }
    nblk_c[c] = run;
  }
  __syncthreads();
  int pos = s_cnt[t];
  for (int b = b0; b < b1; ++b) {
    if (m[b]) {
      if (pos < kCMaxBlk) blist[(int64_t)c * kCMaxBlk + pos] = (uint16_t)b;
      bpos[(int64_t)c * nblk + b] = (uint16_t)min(pos, 65535);
      ++pos;
    } else {
      bpos[(int64_t)c * nblk + b] = 0xffffu;
    }
  }
}

// k_tdens_rows for FP64 with compact, double-buffered staging; same products
// in the same order, so the same partials bit for bit.
__global__ void __launch_bounds__(512) k_tdens_rows_c(TRArgs a, const uint16_t* __restrict__ bpos,
                                                      const uint16_t* __restrict__ blist,
                                                      const int* __restrict__ nblk_c, int nblk,
                                                      uint32_t pairs_off) {
  if (a.sel && *a.sel != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[8];
  const int M = a.M;
  const uint32_t amask = (1u << M) - 1u;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b = blockIdx.x, xcd = b & 7, jj = b >> 3;
  const int slot = (jj / a.nchunk) * 8 + xcd;
  const int chunk = jj % a.nchunk;
  if (slot >= a.n_eb + a.n_id) return;
  const int col = chunk * nt + tid;
  const bool live = col < a.da;
  const uint32_t s = live ? a.astr[col] : a.astr[0];
  const int nb = nblk_c[chunk];
  const uint16_t* bp = bpos + (int64_t)chunk * nblk;
  const uint32_t rbase = lds_addr(smem);
  // alpha sources as ranks (pad = da), then as byte addresses in buffer 0;
  // unused slots read the zero slot after the staged blocks
  uint32_t ex[64];
  int ns = 0;
  alpha_sources<double>(s, amask, a.arank, (uint32_t)a.da * 8u, ex, &ns);
  const uint32_t zslot = rbase + (uint32_t)nb * 16u;
#pragma unroll
  for (int x = 0; x < 64; ++x) {
    const uint32_t r = ex[x] >> 3;
    const bool real = live && r < (uint32_t)a.da;
    const uint32_t pos = bp[(real ? r : 0u) >> 1];  // unconditional: the 64 reads go out together
    ex[x] = real ? rbase + pos * 16u + (r & 1u) * 8u : zslot;
  }
  const uint32_t own = live ? rbase + (uint32_t)bp[col >> 1] * 16u + ((uint32_t)col & 1u) * 8u : zslot;
  int blk[kCPerThread];
#pragma unroll
  for (int k = 0; k < kCPerThread; ++k) {
    const int i = k * nt + tid;
    blk[k] = i < nb ? (int)blist[(int64_t)chunk * kCMaxBlk + i] : 0;
  }
  double acc[64];
#pragma unroll
  for (int x = 0; x < 64; ++x) acc[x] = 0.0;
  double acc_id = 0.0;
  const bool ident = slot >= a.n_eb;
  const int row0 = ident ? (slot - a.n_eb) * a.Kid : 0;
  int nrows;
  if (ident)
    nrows = a.idrows ? max(0, min(a.Kid, *a.n_idrows - row0)) : min(a.Kid, a.db - row0);
  else
    nrows = a.rcount ? a.rcount[slot] : a.K;
  const double* psi = (const double*)a.psi;
  const double* sig = (const double*)a.sig;
  if (tid == 0) {
    *(__attribute__((address_space(3))) double*)(uintptr_t)zslot = 0.0;
    *(__attribute__((address_space(3))) double*)(uintptr_t)(zslot + kCBuf1) = 0.0;
  }
  // the slot's row pairs, copied once into LDS after the two buffers: a
  // pair is then one broadcast LDS read rather than a global load whose
  // latency would sit in front of every copy
  {
    const int2* rl = a.rows + (int64_t)(ident ? 0 : slot) * a.K;
    int2* s_pairs = (int2*)(smem + pairs_off);
    for (int k = tid; k < nrows; k += nt) {
      int2 v;
      if (!ident) {
        v = rl[k];
      } else {
        const int r = a.idrows ? a.idrows[row0 + k] : row0 + k;
        v = make_int2(r, r);
      }
      s_pairs[k] = v;
    }
  }
  __syncthreads();
  const uint32_t s_pairs_addr = rbase + pairs_off;
  auto pair_at = [&](int k) -> int2 {
    const uint64_t u = lds_load<uint64_t>(s_pairs_addr + (uint32_t)k * 8u);
    return make_int2((int)(uint32_t)u, (int)(uint32_t)(u >> 32));
  };
  // pairs k (being formed) and k + 1 (being copied); sv of pair k
  int2 p0 = nrows > 0 ? pair_at(0) : make_int2(0, 0);
  int2 p1 = nrows > 1 ? pair_at(1) : p0;
  double sv0 = (live && nrows > 0) ? sig[(int64_t)(p0.y & 0x7fffffff) * a.da + col] : 0.0;
  if (nrows > 0) stage_blocks(rbase, psi + (int64_t)p0.x * a.da, blk, nb, tid, nt);
  auto step = [&](auto boffc, int k) {
    constexpr uint32_t kOff = decltype(boffc)::value;
    constexpr uint32_t kNext = kOff ? 0u : kCBuf1;
    const int2 p2 = (k + 2 < nrows) ? pair_at(k + 2) : p1;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // sv0 arrived with that wait; passing it through an asm statement keeps
    // the compiler from waiting on its load after the copy below is issued
    // (the hardware counter would then also wait for the copy)
    asm volatile("" : "+v"(sv0));
    __syncthreads();  // pair k staged by every wave; pair k - 1's reads of the other buffer done
    double sv1 = 0.0;
    if (k + 1 < nrows) {
      sv1 = live ? sig[(int64_t)(p1.y & 0x7fffffff) * a.da + col] : 0.0;
      stage_blocks(rbase + kNext, psi + (int64_t)p1.x * a.da, blk, nb, tid, nt);
    }
    if (live) {
      const double w = (p0.y < 0 ? -1.0 : 1.0) * sv0;
#pragma unroll
      for (int g8 = 0; g8 < 8; ++g8) {
        if (g8 * 8 < a.nsx) {
          double v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) v[j] = lds_load<double>(ex[g8 * 8 + j] + kOff);
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[g8 * 8 + j] += w * v[j];
        }
      }
      if (!ident) acc_id += w * lds_load<double>(own + kOff);
    }
    p0 = p1;
    p1 = p2;
    sv0 = sv1;
  };
  int k = 0;
  for (; k + 1 < nrows; k += 2) {
    step(std::integral_constant<uint32_t, 0u>(), k);
    step(std::integral_constant<uint32_t, kCBuf1>(), k + 1);
  }
  if (k < nrows) step(std::integral_constant<uint32_t, 0u>(), k);
  // flush, as in k_tdens_rows
  __syncthreads();
  double* s_bins = (double*)smem;  // [nt / 64][kBins]
  const int nw = nt >> 6;
  for (int i = tid; i < nw * kBins; i += nt) s_bins[i] = 0.0;
  __syncthreads();
  if (live) {
    uint32_t bins[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) bins[x] = 0u;
    uint64_t signs = 0;
    alpha_bins(s, amask, bins, &signs);
    if (!a.fsign) signs = 0;
#pragma unroll
    for (int x = 0; x < 64; ++x) {
      if (x < ns) {
        const uint32_t bin = (bins[x >> 2] >> ((x & 3) * 8)) & 0xffu;
        atomicAdd(&s_bins[(tid >> 6) * kBins + bin], ((signs >> x) & 1ull) ? -acc[x] : acc[x]);
      }
    }
  }
  double d = acc_id;
  for (int o = 32; o > 0; o >>= 1) d += __shfl_down(d, o, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = d;
  __syncthreads();
  double* out = a.part + ((int64_t)slot * a.nchunk + chunk) * kStageW;
  for (int x = tid; x < kBins; x += nt) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_bins[w * kBins + x];
    out[x] = t;
  }
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += s_red[w];
    out[kBins] = t;
  }
}

// Fixed-order sums of the row-batched partials:
//   Tab[ea][eb] = sum over chunks of slot eb's bin ea,  Tb[eb] = the same of
//   its identity bin,  Ta[ea] = sum over the identity slices and chunks.
__global__ void k_tdens_rows_final(const double* part, int n_eb, int n_id, int nchunk, double* Ta, double* Tb,
                                   double* Tab, const int* sel) {
  if (sel && *sel != 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBins * kStageW) {
    const int eb = i / kStageW, x = i % kStageW;
    double t = 0.0;
    if (eb < n_eb)
      for (int c = 0; c < nchunk; ++c) t += part[((int64_t)eb * nchunk + c) * kStageW + x];
    if (x < kBins) Tab[(int64_t)x * kBins + eb] = t;
    else Tb[eb] = t;
  } else if (i < kBins * kStageW + kBins) {
    const int x = i - kBins * kStageW;
    double t = 0.0;
    for (int sl = 0; sl < n_id; ++sl)
      for (int c = 0; c < nchunk; ++c) t += part[((int64_t)(n_eb + sl) * nchunk + c) * kStageW + x];
    Ta[x] = t;
  }
}

// ------------------------------------------ transition values on matrix cores
//
// The singles and alpha-beta doubles of the sweep per target beta row I_b
// as dense products.  Stage the row's kept beta-single sources J_k (k < 64,
// ordered beta excitation eb_k from J_k to I_b, pool sign s_k) as
// P[k][t] = psi[J_k][t] and the target row sigma[I_b][.] whole in LDS.  For
// alpha orbital e (wave e) and source strings t holding e,
//   X_e[i][k] = sum_t A_e[i][t] P[k][t],
//   A_e[i][t] = (alpha pool sign of (i, e) at s) sigma[I_b][s],  s = t - e + i,
// is a (16 x n) x (n x 64) product on v_mfma_f64_16x16x4_f64 (A operand:
// lane l row i = l & 15, column t of step slot l >> 4; B operand: stage
// k = 16 b + (l & 15) of the same column), and
//   Tab[(i, e)][eb_k] += s_k X_e[i][k]  (i empty in t),
//   Tb[eb_k] += s_k X_e[e][k]  (row i = e: A = sigma[I_b][t], counted at the
//               lowest occupied orbital of t only, so each t once; the empty
//               string, which has none, at orbital 0),
//   Ta[(i, e)] += sum_t A_e[i][t] psi[I_b][t]  (the row's own amplitudes).
// Each of kTMWG persistent workgroups adds its rows into a partial table of
// its own, every entry of which only one wave touches, rows in a fixed
// order, a row's additions complete before the next row's; a fixed-order
// pass sums the partials: the results are reproducible bit for bit.
constexpr int kTMSeg = 16;                 // columns per segment
constexpr int kTMSegs = 3;                 // segments per chunk, from three regions of the alpha space
constexpr int kTMCols = kTMSeg * kTMSegs;  // columns per chunk
constexpr int kTMLd = kTMCols + 1;         // staged row stride: a column read by 16 stages hits 16 bank pairs
constexpr int kTMWG = 256;                 // persistent workgroups
constexpr int kTMPart = kBins * kBins + kBins + 16 * kBins;  // partial: Tab | Ta | Tb per orbital
__host__ __device__ inline int tm_column(int c, int l, int qr) {
  return (l / kTMSeg) * qr + c * kTMSeg + l % kTMSeg;
}

template <typename T>
struct TMLds {
  T P[2][65][kTMLd];          // rows < 64: kept beta-single sources (zero past them); row 64: the own row
  uint32_t lst[16][kTMCols];  // per wave: chunk column | alpha string << 8, columns with its orbital occupied
  int32_t rlo[256], rhi[256]; // alpha rank tables
  int2 stage[64];             // (source rank, eb | pool sign << 16)
  int nstage;
  int own;
};

struct TMArgs {
  const void* psi;
  const void* sig;
  const int* sel;          // device-side choice under support skipping: runs where *sel == 1 (null: always)
  int M, nb, da, db, qr, nch;
  const uint32_t* astr;
  const RankTables* arank;
  const uint32_t* bstr;
  const RankTables* brank;
  const uint32_t* row_nz;  // support flags of psi's beta rows, or null
  double* part;            // [gridDim][kTMPart]
  int fsign;
};

template <typename T>
__global__ void __launch_bounds__(1024) k_tdens_m(TMArgs a) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) TMLds<T> L;
  T* srow = (T*)smem;  // [da]: the target row of sigma
  const int M = a.M, da = a.da;
  const uint32_t bmask = (1u << M) - 1u;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int e = w;
  const bool ew = e < M;
  if (a.sel && *a.sel != 1) return;
  double* part = a.part + (size_t)blockIdx.x * kTMPart;
  double* pTa = part + kBins * kBins;
  double* pTb = pTa + kBins;
  for (int x = tid; x < kTMPart; x += 1024) part[x] = 0.0;
  if (tid < 256) {
    L.rlo[tid] = a.arank->lo[tid];
    L.rhi[tid] = a.arank->hi[tid];
  }
  const T* psi = (const T*)a.psi;
  const T* sig = (const T*)a.sig;
  // staging pieces: 4 bytes, kPPR per row, 64 per copy, kIPR copies per row
  constexpr int kPPR = kTMCols * (int)sizeof(T) / 4;
  constexpr int kIPR = (kPPR + 63) / 64;
  constexpr int kNI = 65 * kIPR;  // copies per buffer
  int gpart[kIPR];                // chunk-0 column of the lane's piece in part j of a row, -1 past the row
  int wpart[kIPR];                // byte within the element
#pragma unroll
  for (int j = 0; j < kIPR; ++j) {
    const int piece = j * 64 + lane;
    const int lb = piece * 4;
    gpart[j] = piece < kPPR ? tm_column(0, lb / (int)sizeof(T), a.qr) : -1;
    wpart[j] = lb % (int)sizeof(T);
  }
  const int i_a = lane & 15;  // A-operand row
  // pair bin of (i_a, e), and the orbitals strictly between them
  const int pbin = (max(i_a, e) * (max(i_a, e) - 1) / 2 + min(i_a, e)) * 2 + (i_a > e ? 1 : 0);
  const uint32_t btw = (i_a < M && i_a != e && ew) ? betw(min(i_a, e), max(i_a, e)) : 0u;
  // target of (i_a, e) from t: t ^ flip (t itself for i_a = e)
  const uint32_t flip = (i_a == e) ? 0u : (1u << e) ^ (1u << i_a);
  const uint32_t diag = (i_a == e) ? 1u : 0u;
  const uint32_t lane_ok = (ew && i_a < M) ? 1u : 0u;
  const uint32_t ebit = 1u << e, ibit = 1u << i_a;
  // alpha string of chunk column `lane` | 1 << 31 (0 past the columns)
  auto string_of = [&](int c) -> uint32_t {
    const int g = tm_column(c, lane, a.qr);
    return (lane < kTMCols && g < da) ? (a.astr[g] | 0x80000000u) : 0u;
  };
  for (int brow = blockIdx.x; brow < a.db; brow += gridDim.x) {
    __syncthreads();  // the previous row is done with the staging buffers and the sigma row
    const uint32_t bs = a.bstr[brow];
    const int nbemp = M - a.nb, nbs = a.nb * nbemp;
    if (tid < 64) {
      const int jb = tid;
      bool keep = false;
      int2 ent = make_int2(0, 0);
      if (jb < nbs) {
        const int io = jb / nbemp, ie = jb % nbemp;
        uint32_t occ = bs, emp = ~bs & bmask;
        for (int j = 0; j < io; ++j) occ &= occ - 1;
        for (int j = 0; j < ie; ++j) emp &= emp - 1;
        const int i = __ffs(occ) - 1, ee = __ffs(emp) - 1;
        const int p = min(i, ee), q = max(i, ee);
        const uint32_t src = bs ^ (1u << i) ^ (1u << ee);
        const int eb = (q * (q - 1) / 2 + p) * 2 + (i == q ? 1 : 0);
        const uint32_t sg = __popc(betw(p, q) & src) & (uint32_t)a.fsign;
        const int r2 = a.brank->lo[src & 255u] + a.brank->hi[(src >> 8) & 255u];
        ent = make_int2(r2, eb | (int)(sg << 16));
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
    if (nst == 0 && !own) continue;
    const int nblk = (nst + 15) >> 4;  // 16-stage MFMA blocks
    for (int x = tid; x < 2 * 65 * kTMLd; x += 1024) {
      const int r = (x / kTMLd) % 65;
      if ((r >= nst && r < 64) || (r == 64 && !own)) (&L.P[0][0][0])[x] = T(0);
    }
    // the sigma row (its copies complete before the barrier of chunk 0)
    stage_row_lds(srow, sig + (int64_t)brow * da, da * (int)sizeof(T), tid, 1024);
    auto issue = [&](int c, int bf) {
      for (int ins = w; ins < kNI; ins += 16) {
        const int row = ins / kIPR, j = ins % kIPR;
        if (row < nst || (row == 64 && own)) {
          const int src = row == 64 ? brow : L.stage[row].x;
          const uint32_t dst =
              (uint32_t)__builtin_amdgcn_readfirstlane(lds_addr(&L.P[bf][row][0]) + (uint32_t)j * 256u);
          int gp = -1;
          int wp = 0;
#pragma unroll
          for (int jj = 0; jj < kIPR; ++jj)
            if (jj == j) {
              gp = gpart[jj];
              wp = wpart[jj];
            }
          const int g = gp + c * kTMSeg;
          if (gp >= 0 && g < da) dma4(dst, (const char*)(psi + (int64_t)src * da + g) + wp);
        }
      }
    };
    f64x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    double oacc = 0.0;
    const uint32_t srow_a = lds_addr(srow);
    uint32_t tv = string_of(0);
    issue(0, 0);
    for (int c = 0; c < a.nch; ++c) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // chunk c in its buffer; every wave done with chunk c - 1
      uint32_t tvn = 0u;
      if (c + 1 < a.nch) {
        tvn = string_of(c + 1);
        issue(c + 1, (c + 1) & 1);
      }
      // the wave's columns with its orbital occupied (wave 0 also takes the
      // empty string)
      const uint32_t tc = tv & 0xffffu;
      const bool bit = ew && (tv >> 31) && (((tc >> e) & 1u) || (tc == 0u && e == 0));
      const uint64_t m = __ballot(bit);
      const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      if (bit) L.lst[w][__popcll(m & below)] = (uint32_t)lane | (tc << 8);
      const int n = __popcll(m);
      tv = tvn;
      const uint32_t pb = lds_addr(&L.P[c & 1][i_a][0]);  // stage i_a of block 0
      const uint32_t po = lds_addr(&L.P[c & 1][64][0]);   // the own row
      const int nsteps = (n + 3) >> 2;
      // one step: the A element (sigma at the target of (i_a, e) from the
      // column's string t, with its sign; zero where there is none) and the
      // B operands of the column, all of whose reads wait only for the list
      // one step: the A element (sigma at the target of (i_a, e) from the
      // column's string t, with its sign; zero where there is none) and the
      // B operands of the column, all of whose reads wait only for the list
      // entry, which is read a step ahead.  The element's validity is formed
      // without branches from the lane's masks.
      auto entry = [&](int st) -> uint32_t {
        const int slot = 4 * st + (lane >> 4);
        return L.lst[w][slot < n ? slot : 0] | (slot < n ? 0x80000000u : 0u);
      };
      auto step = [&](uint32_t cur, auto full) {
        constexpr bool kFull = decltype(full)::value;
        const uint32_t cl = cur & 63u;
        const uint32_t t = (cur >> 8) & 0xffffu;
        const uint32_t s2 = t ^ flip;
        const uint32_t low = t ? (uint32_t)(__ffs(t) - 1) : 0u;  // lowest occupied orbital (0 for the empty string)
        const uint32_t ok = (cur >> 31) & lane_ok &
                            ((diag & (uint32_t)(low == (uint32_t)e)) |
                             ((diag ^ 1u) & (uint32_t)((t & ebit) != 0u) & (uint32_t)((t & ibit) == 0u)));
        const int r0 = L.rlo[s2 & 255u] + L.rhi[(s2 >> 8) & 255u];  // any byte indexes the tables
        double bv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
          bv[b] = (double)lds_load<T>(pb + (uint32_t)(16 * b * kTMLd + (int)cl) * (uint32_t)sizeof(T));
        const double pw = own ? (double)lds_load<T>(po + cl * (uint32_t)sizeof(T)) : 0.0;
        const double v = (double)lds_load<T>(srow_a + (uint32_t)(ok ? r0 : 0) * (uint32_t)sizeof(T));
        const double sv = ((__popc(btw & s2) & a.fsign) != 0) ? -v : v;
        const double av = ok ? sv : 0.0;
        oacc += av * pw;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (kFull || b < nblk) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[b], acc[b], 0, 0, 0);
      };
      uint32_t ent = entry(0);
      // (rows past the kept stages are zero: their reads are harmless; the
      // products of whole blocks past them are skipped)
#pragma unroll 1
      for (int st = 0; st < nsteps; ++st) {
        const uint32_t cur = ent;
        ent = entry(st + 1);
        step(cur, std::integral_constant<bool, false>());
      }
    }
    // the row's values into the partial (element q of lane l: row
    // (l >> 4) + 4q, stage 16 b + (l & 15))
    oacc += __shfl_xor(oacc, 16, 64);
    oacc += __shfl_xor(oacc, 32, 64);
    if (ew) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 16 * b + (lane & 15);
        if (b < nblk && k < nst) {
          const int info = L.stage[k].y;
          const int eb = info & 0xffff;
          const bool neg = (info >> 16) & 1;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = (lane >> 4) + 4 * q;
            const double v = neg ? -acc[b][q] : acc[b][q];
            if (i == e)
              unsafeAtomicAdd(pTb + e * kBins + eb, v);
            else if (i < M)
              unsafeAtomicAdd(part + (size_t)((max(i, e) * (max(i, e) - 1) / 2 + min(i, e)) * 2 + (i > e ? 1 : 0)) *
                                         kBins + eb,
                              v);
          }
        }
      }
      if (own && lane < M && lane != e) unsafeAtomicAdd(pTa + pbin, oacc);
    }
  }
}

// Fixed-order sums of the workgroups' partials.
__global__ void k_tm_final(const double* __restrict__ part, int nwg, double* Ta, double* Tb, double* Tab,
                           const int* sel) {
  if (sel && *sel != 1) return;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < kBins * kBins) {
    double t = 0.0;
    for (int g = 0; g < nwg; ++g) t += part[(size_t)g * kTMPart + x];
    Tab[x] = t;
  } else if (x < kBins * kBins + kBins) {
    const int ea = x - kBins * kBins;
    double t = 0.0;
    for (int g = 0; g < nwg; ++g) t += part[(size_t)g * kTMPart + kBins * kBins + ea];
    Ta[ea] = t;
  } else if (x < kBins * kBins + 2 * kBins) {
    const int eb = x - kBins * kBins - kBins;
    double t = 0.0;
    for (int g = 0; g < nwg; ++g)
      for (int e = 0; e < 16; ++e) t += part[(size_t)g * kTMPart + kBins * kBins + kBins + e * kBins + eb];
    Tb[eb] = t;
  }
}

// Under support skipping: the matrix-core form where at least a quarter of
// the beta rows hold amplitude (*sel = 1), else the row-batched kernel,
// whose work follows the kept row pairs (*sel = 0).
__global__ void __launch_bounds__(1024) k_tm_select(const uint32_t* __restrict__ flags, int nrow, int* __restrict__ sel) {
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

// (source row, target row | sign << 31) of every ordered beta single
// excitation eb = (created ci, annihilated ae): source rows hold ae and not
// ci, in colex order over the other orbitals.  One thread per (eb, k).
__global__ void k_eb_rows(int M, int nb, int n_eb, int K, const RankTables* brank, int fsign, int2* rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_eb * K) return;
  const int eb = (int)(i / K), k = (int)(i % K);
  const int pid = eb >> 1, O = eb & 1;
  int q = 1;
  while ((q + 1) * q / 2 <= pid) ++q;
  const int p = pid - q * (q - 1) / 2;
  const int ci = O ? q : p, ae = O ? p : q;
  const uint32_t freem = ((1u << M) - 1u) & ~((1u << ci) | (1u << ae));
  const int nfree = M - 2, nsel = nb - 1;
  uint32_t pos = 0;
  int rr = k;
  for (int j = nsel; j >= 1; --j) {
    int c = j - 1;
    while (c + 1 < nfree && c_binom_s[c + 1][j] <= rr) ++c;
    rr -= c_binom_s[c][j];
    pos |= 1u << c;
  }
  uint32_t src = 1u << ae, f = freem;
  for (int bb = 0; f; ++bb) {
    const uint32_t low = f & (~f + 1u);
    if (pos & (1u << bb)) src |= low;
    f ^= low;
  }
  const uint32_t tgt = src ^ (1u << ci) ^ (1u << ae);
  const uint32_t sg = __popc(betw(p, q) & src) & (uint32_t)fsign;
  const int rs = brank->lo[src & 255u] + brank->hi[(src >> 8) & 255u];
  const int rt = brank->lo[tgt & 255u] + brank->hi[(tgt >> 8) & 255u];
  rows[i] = make_int2(rs, (int)((uint32_t)rt | (sg << 31)));
}

// Fixed-order sums of the partials, two levels (both deterministic).
//   Ta[ea]      = sum over rows and chunks of the stage-0 bins
//   Tab[ea][eb] = sum over the target rows holding the ordered beta excitation
//                 eb (created orbital occupied, annihilated one empty) of that
//                 row's stage for eb;  Tb[eb] = the same rows' beta-single bin
constexpr int kRowSlices = 16;
constexpr int kRowBlocks = 256;

// grid (kBins, kRowSlices): partial sums of Tab[.][eb] and Tb[eb] over a slice
// of the target rows of eb
__global__ void k_tdens_reduce_ab(TArgs a, double* red) {
  const int eb = blockIdx.x, slice = blockIdx.y;
  const int tid = threadIdx.x;
  const int M = a.M;
  const int x0 = tid, x1 = tid + blockDim.x;
  double acc0 = 0.0, acc1 = 0.0;
  const int pid = eb >> 1, O = eb & 1;
  int q = 1;
  while ((q + 1) * q / 2 <= pid) ++q;
  const int p = pid - q * (q - 1) / 2;
  if (q < M) {
    const int ci = O ? q : p, ae = O ? p : q;  // created (occupied in target), annihilated
    const int nbemp = M - a.nb;
    const uint32_t freem = ((1u << M) - 1u) & ~((1u << ci) | (1u << ae));
    const int nfree = M - 2, nsel = a.nb - 1;
    const int nrows = (nsel < 0 || nsel > nfree) ? 0 : c_binom_s[nfree][nsel];
    const int r0 = (int)((int64_t)nrows * slice / kRowSlices), r1 = (int)((int64_t)nrows * (slice + 1) / kRowSlices);
    for (int r = r0; r < r1; ++r) {
      uint32_t pos = 0;
      int rr = r;
      for (int j = nsel; j >= 1; --j) {
        int c = j - 1;
        while (c + 1 < nfree && c_binom_s[c + 1][j] <= rr) ++c;
        rr -= c_binom_s[c][j];
        pos |= 1u << c;
      }
      uint32_t str = 1u << ci, f = freem;
      for (int bb = 0; f; ++bb) {
        const uint32_t low = f & (~f + 1u);
        if (pos & (1u << bb)) str |= low;
        f ^= low;
      }
      const int row = a.brank->lo[str & 255u] + a.brank->hi[(str >> 8) & 255u];
      const int io = __popc(str & ((1u << ci) - 1u));
      const int ie = __popc(~str & ((1u << ae) - 1u));
      const int stg = 1 + io * nbemp + ie;
      const double* pp = a.part + (((int64_t)row * a.nchunk) * a.nstage + stg) * kStageW;
      const int64_t cstride = (int64_t)a.nstage * kStageW;
      for (int c = 0; c < a.nchunk; ++c) {
        if (x0 < kStageW) acc0 += pp[c * cstride + x0];
        if (x1 < kStageW) acc1 += pp[c * cstride + x1];
      }
    }
  }
  double* o = red + ((int64_t)eb * kRowSlices + slice) * kStageW;
  if (x0 < kStageW) o[x0] = acc0;
  if (x1 < kStageW) o[x1] = acc1;
}

// grid kRowBlocks: partial sums of the stage-0 bins over a block of rows
__global__ void k_tdens_reduce_a(TArgs a, double* red) {
  const int blk = blockIdx.x;
  const int r0 = (int)((int64_t)a.db * blk / kRowBlocks), r1 = (int)((int64_t)a.db * (blk + 1) / kRowBlocks);
  for (int x = threadIdx.x; x < kBins; x += blockDim.x) {
    double t = 0.0;
    for (int r = r0; r < r1; ++r)
      for (int c = 0; c < a.nchunk; ++c) t += a.part[(((int64_t)r * a.nchunk + c) * a.nstage) * kStageW + x];
    red[(int64_t)blk * kBins + x] = t;
  }
}

__global__ void k_tdens_final(const double* red_ab, const double* red_a, double* Ta, double* Tb, double* Tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBins * kStageW) {
    const int eb = i / kStageW, x = i % kStageW;
    double t = 0.0;
    for (int sl = 0; sl < kRowSlices; ++sl) t += red_ab[((int64_t)eb * kRowSlices + sl) * kStageW + x];
    if (x < kBins) Tab[(int64_t)x * kBins + eb] = t;
    else Tb[eb] = t;
  } else if (i < kBins * kStageW + kBins) {
    const int x = i - kBins * kStageW;
    double t = 0.0;
    for (int b = 0; b < kRowBlocks; ++b) t += red_a[(int64_t)b * kBins + x];
    Ta[x] = t;
  }
}

__device__ inline int ord_bin(uint32_t cre, uint32_t ann) {  // one-spin single: created, annihilated
  const int c = __ffs(cre) - 1, e = __ffs(ann) - 1;
  const int p = min(c, e), q = max(c, e);
  return (q * (q - 1) / 2 + p) * 2 + (c == q ? 1 : 0);
}

// grad[k] for singles and alpha-beta doubles from the transition values;
// same-spin doubles were written by k_gram_grad.
__global__ void k_tdens_grad(const hyp_exc* ops, int64_t n, int M, const double* Ta, const double* Tb,
                             const double* Tab, double* grad, int* bad_rec) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t m = (1u << M) - 1u;
  const hyp_exc op = ops[k];
  const int bad = exc_status(op, M);
  if (bad != HYP_OK) {  // an invalid excitation: NaN, nothing indexed
    grad[k] = __builtin_nan("");
    note_bad_exc(bad_rec, bad, k);
    return;
  }
  const uint32_t ca = op.cre & m, aa = op.ann & m, cb = (op.cre >> M) & m, ab = (op.ann >> M) & m;
  const int na_ = __popc(ca), nb_ = __popc(cb);
  double g;
  if (na_ == 1 && nb_ == 0) {
    const int e = ord_bin(ca, aa);
    g = 2.0 * (Ta[e] - Ta[e ^ 1]);
  } else if (na_ == 0 && nb_ == 1) {
    const int e = ord_bin(cb, ab);
    g = 2.0 * (Tb[e] - Tb[e ^ 1]);
  } else if (na_ == 1 && nb_ == 1) {
    const int ea = ord_bin(ca, aa), eb = ord_bin(cb, ab);
    g = 2.0 * (Tab[(int64_t)ea * kBins + eb] - Tab[(int64_t)(ea ^ 1) * kBins + (eb ^ 1)]);
  } else {
    return;  // same-spin double: k_gram_grad
  }
  grad[k] = g;
}

__device__ inline uint32_t gram_string(uint32_t cm, uint32_t am, int M, int N, int i) {
  // i-th string (colex over the free orbitals) holding am and not cm
  const uint32_t freem = ((1u << M) - 1u) & ~(cm | am);
  const int nfree = __popc(freem), nsel = N - __popc(am);
  uint32_t pos = 0;
  int r = i;
  for (int j = nsel; j >= 1; --j) {
    int c = j - 1;
    while (c + 1 < nfree && c_binom_s[c + 1][j] <= r) ++c;
    r -= c_binom_s[c][j];
    pos |= 1u << c;
  }
  uint32_t s = am, f = freem;
  for (int b = 0; f; ++b) {
    const uint32_t low = f & (~f + 1u);
    if (pos & (1u << b)) s |= low;
    f ^= low;
  }
  return s;
}

__device__ inline int gram_sign(uint32_t cm, uint32_t am, uint32_t s) {
  int odd = 0;
  uint32_t a = am;
  while (a) {
    const int q = __ffs(a) - 1;
    a &= a - 1;
    odd += __popc(s & ((1u << q) - 1u));
    s ^= 1u << q;
  }
  uint32_t c = cm;
  while (c) {
    const int q = 31 - __clz(c);
    c ^= 1u << q;
    odd += __popc(s & ((1u << q) - 1u));
    s ^= 1u << q;
  }
  return odd & 1;
}

// Colex rank of a core (a k-subset) and the slot of a 2-orbital mask among
// the pairs of the orbitals outside it (comp): w (w - 1) / 2 + u for the
// mask's orbitals at positions u < w of comp, as the core Gram blocks are
// laid out.
__device__ inline int core_rank(uint32_t K) {
  int r = 0, j = 0;
  while (K) {
    const int o = __ffs(K) - 1;
    K &= K - 1;
    r += c_binom_s[o][++j];
  }
  return r;
}
__device__ inline int core_slot(uint32_t comp, uint32_t m2) {
  const int p = __ffs(m2) - 1, q = 31 - __clz(m2);
  const int u = __popc(comp & ((1u << p) - 1u)), w = __popc(comp & ((1u << q) - 1u));
  return w * (w - 1) / 2 + u;
}

// One workgroup per generator: same-spin doubles get
// g = 2 sum_J s (Gc[tau J][J] - Gc[J][tau J]) over the generator's strings J,
// read from the block of the core K = J - {a1, a2} (Gc[K][i][j] = sum over
// the other spin of sigma(slot i) psi(slot j)); other generators are skipped.
__global__ void k_gram_grad(const hyp_exc* ops, int M, int na, int nb, const double* Ga, int Sa, const double* Gb,
                            int Sb, int fsign, double* grad) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  const uint32_t m = (1u << M) - 1u;
  const hyp_exc op = ops[k];
  if (exc_status(op, M) != HYP_OK) return;  // k_tdens_grad writes NaN
  const int ca = __popc(op.cre & m), cb = __popc((op.cre >> M) & m);
  const bool alpha = ca == 2 && cb == 0, beta = ca == 0 && cb == 2;
  if (!alpha && !beta) return;
  const uint32_t cm = alpha ? (op.cre & m) : ((op.cre >> M) & m);
  const uint32_t am = alpha ? (op.ann & m) : ((op.ann >> M) & m);
  const int N = alpha ? na : nb;
  const double* G = alpha ? Ga : Gb;
  const int64_t S = alpha ? Sa : Sb;
  const int nfree = M - 4, nsel = N - 2;
  const int cnt = (nsel < 0 || nsel > nfree) ? 0 : c_binom_s[nfree][nsel];
  double acc = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const uint32_t J = gram_string(cm, am, M, N, i);
    const uint32_t core = J & ~am;
    const uint32_t comp = m & ~core;
    const double* Gk = G + (int64_t)core_rank(core) * S * S;
    const int64_t sI = core_slot(comp, cm), sJ = core_slot(comp, am);
    const double v = Gk[sI * S + sJ] - Gk[sJ * S + sI];
    acc += (gram_sign(cm, am, J) & fsign) ? -v : v;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) grad[k] = 2.0 * (red[0] + red[1] + red[2] + red[3]);
}

// ---------------------------------------------------------------- support

__global__ void k_zero_u32(uint32_t* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Row and column support of m[rows][cols] (flags cleared beforehand): 64x64
// tiles, a wave per row of the tile (ballot), each lane keeps its column's
// flag over the tile's rows.
template <typename T>
__global__ void __launch_bounds__(256) k_support(const T* __restrict__ m, int rows, int cols,
                                                 uint32_t* __restrict__ row_nz, uint32_t* __restrict__ col_nz) {
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int cc = c0 + tx;
  bool cany = false;
  for (int r = ty; r < 64; r += 4) {
    const int rr = r0 + r;
    bool nz = false;
    if (rr < rows && cc < cols) nz = m[(int64_t)rr * cols + cc] != T(0);
    cany |= nz;
    if (__ballot(nz) && tx == 0) row_nz[rr] = 1u;
  }
  if (cany) col_nz[cc] = 1u;
}

// Ordered list of the indices i < n with flag[i] != 0, and its length: one
// workgroup of 1024 threads, 1024 flags per round.
__global__ void __launch_bounds__(1024) k_list_nz(const uint32_t* __restrict__ flag, int n, int* __restrict__ list,
                                                  int* __restrict__ count) {
  __shared__ int s_wc[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int b0 = 0; b0 < n; b0 += 1024) {
    const int i = b0 + tid;
    const bool f = i < n && flag[i] != 0u;
    const uint64_t m = __ballot(f);
    if (lane == 0) s_wc[w] = __popcll(m);
    __syncthreads();
    int off = s_base;
    for (int j = 0; j < w; ++j) off += s_wc[j];
    if (f) list[off + __popcll(m & below)] = i;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int j = 0; j < 16; ++j) t += s_wc[j];
      s_base += t;
    }
    __syncthreads();
  }
  if (tid == 0) *count = s_base;
}

// Row pairs of each beta excitation whose source row is in psi's support,
// in order, at the front of the excitation's K slots; rcount[eb] their
// number.  One wave per beta excitation.
__global__ void __launch_bounds__(256) k_rows_compact(const int2* __restrict__ rows, int n_eb, int K,
                                                      const uint32_t* __restrict__ row_nz,
                                                      int2* __restrict__ crows, int* __restrict__ rcount) {
  const int eb = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (eb >= n_eb) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)eb * K;
  int n = 0;
  for (int k0 = 0; k0 < K; k0 += 64) {
    const int k = k0 + lane;
    int2 rp = make_int2(0, 0);
    bool keep = false;
    if (k < K) {
      rp = rows[base + k];
      keep = row_nz[rp.x] != 0u;
    }
    const uint64_t m = __ballot(keep);
    if (keep) crows[base + n + __popcll(m & below)] = rp;
    n += __popcll(m);
  }
  if (lane == 0) rcount[eb] = n;
}

namespace {
struct TScratch {
  double* part = nullptr;
  size_t cap = 0;
  double* T = nullptr;   // Ta | Tb | Tab
  double* red = nullptr; // second-level partials
  bool binom = false;
  double* gram = nullptr;  // core Gram blocks (alpha | beta) | dense FP64 operand rows
  size_t gram_cap = 0;
  int2* rows = nullptr;    // beta excitation row pairs of the row-batched kernel
  int rows_M = -1, rows_nb = -1, rows_fsign = -1;
  size_t rows_cap = 0;
  double* rpart = nullptr; // partials of the row-batched kernel
  size_t rpart_cap = 0;
  // support skipping: flags and ordered lists of psi's nonzero beta rows
  // and alpha columns, their two lengths (device memory: every decision
  // that depends on them is taken on the device), and the kept row pairs of
  // each beta excitation
  uint32_t* nz = nullptr;
  int* lists = nullptr;
  size_t nz_cap = 0;
  int* cnt = nullptr;
  int2* crows = nullptr;
  int* rcount = nullptr;
  size_t crows_cap = 0;
  // compact staging tables of k_tdens_rows_c, one entry per (orbitals,
  // alpha electrons, chunk width) seen on the device (batched sweeps mix
  // string spaces), oldest replaced first; ok: every chunk fits the buffers
  struct CTab {
    uint16_t* bpos = nullptr;
    uint16_t* blist = nullptr;
    int* nb = nullptr;
    int M = -1, na = -1, nt = -1, max = 0;
    bool ok = false;
  };
  CTab ctab[8];
  int ctab_next = 0;
  // matrix-core transition values: the workgroups' partials and the
  // device-side choice of form under support skipping
  double* tm_part = nullptr;
  int* tm_sel = nullptr;
};
TScratch g_ts[64];
}  // namespace
int g_row_staging = 0;  // 0 compact where it applies, 1 whole rows

bool row_staging_compact() { return g_row_staging == 0; }

hyp_status build_compact_tables(const Sector* S, int nt, uint16_t** bpos, uint16_t** blist, int** nb, int* max_nb,
                                hipStream_t st) {
  const int da = (int)S->da, nblk = (da + 1) / 2, nchunk = (da + nt - 1) / nt;
  *bpos = nullptr;
  *blist = nullptr;
  *nb = nullptr;
  *max_nb = 0;
  uint8_t* mark = nullptr;
  const int mwords = (int)(((size_t)nchunk * nblk + 3) / 4);
  hipError_t e = hipMalloc(bpos, (size_t)nchunk * nblk * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(blist, (size_t)nchunk * kCMaxBlk * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(nb, (size_t)nchunk * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&mark, (size_t)mwords * 4);
  std::vector<int> h((size_t)nchunk);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min(1024, (mwords + 255) / 256)), dim3(256), 0, st,
                       (uint32_t*)mark, mwords);
    hipLaunchKernelGGL(k_cs_mark, dim3((unsigned)((da + 255) / 256)), dim3(256), 0, st, da, nt, S->M, S->d_astr,
                       S->d_arank, nblk, mark);
    hipLaunchKernelGGL(k_cs_scan, dim3((unsigned)nchunk), dim3(256), 0, st, mark, nblk, *bpos, *blist, *nb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), *nb, (size_t)nchunk * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (mark) (void)hipFree(mark);
  if (e != hipSuccess) {
    (void)hipFree(*bpos);
    (void)hipFree(*blist);
    (void)hipFree(*nb);
    *bpos = nullptr;
    *blist = nullptr;
    *nb = nullptr;
    return hip_fail(e, "build_compact_tables");
  }
  *max_nb = h.empty() ? 0 : *std::max_element(h.begin(), h.end());
  return HYP_OK;
}

// The sweep's compact staging tables of a string space and chunk width
// (built on first use).
static hyp_status compact_tables(Sector* S, TScratch& ts, int nt, hipStream_t st, const TScratch::CTab** out) {
  for (const TScratch::CTab& t : ts.ctab)
    if (t.M == S->M && t.na == S->na && t.nt == nt) {
      *out = &t;
      return HYP_OK;
    }
  TScratch::CTab& t = ts.ctab[ts.ctab_next];
  if (t.bpos || t.blist || t.nb) {
    HYP_HIP(hipDeviceSynchronize());  // queued launches may still read the replaced entry
    if (t.bpos) HYP_HIP(hipFree(t.bpos));
    if (t.blist) HYP_HIP(hipFree(t.blist));
    if (t.nb) HYP_HIP(hipFree(t.nb));
  }
  t = TScratch::CTab();
  int mx = 0;
  hyp_status r = build_compact_tables(S, nt, &t.bpos, &t.blist, &t.nb, &mx, st);
  if (r != HYP_OK) return r;
  t.max = mx;
  t.ok = mx <= kCMaxBlk && (mx + nt - 1) / nt <= kCPerThread;
  t.M = S->M;
  t.na = S->na;
  t.nt = nt;
  ts.ctab_next = (ts.ctab_next + 1) % 8;
  *out = &t;
  return HYP_OK;
}

size_t tdens_bytes(const Sector* S) {
  const int nt = std::max(64, std::min(768, (int)((S->da + 63) / 64 * 64)));
  const int64_t nchunk = (S->da + nt - 1) / nt;
  const int64_t nstage = 1 + (int64_t)S->nb * (S->M - S->nb);
  return (size_t)S->db * nchunk * nstage * kStageW * sizeof(double);
}

// Full-sweep gradients for the ops list: transition values for singles and
// alpha-beta doubles, Gram matrices for same-spin doubles.
static int64_t binom64(int m, int k) {
  if (k < 0 || k > m) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (m - k + i) / i;
  return r;
}

// The singles and alpha-beta doubles on the matrix cores (k_tdens_m) where
// the target row fits LDS and the mode switch takes them (in auto mode above
// kTMAutoBytes: below, the state stays in the Infinity Cache and the
// row-batched kernel is faster, 5.3 against 7.8 ms at 28 qubits); *done
// false otherwise.
static hyp_status tdens_mm(Sector* S, hyp_dtype dt, TScratch& ts, const void* psi, const void* sig, double* Ta,
                           double* Tb, double* Tab, bool skip, hipStream_t st, bool* done, const int** sel) {
  *done = false;
  *sel = nullptr;
  const int mode = mixed_mm_mode();
  const int M = S->M, na = S->na, da = (int)S->da, db = (int)S->db;
  const size_t tsz = dt == HYP_F64 ? 8 : 4;
  const size_t lds = (size_t)da * tsz + (tsz == 8 ? sizeof(TMLds<double>) : sizeof(TMLds<float>));
  if (mode == 0 || M > kMaxOrb || da <= 0 || db <= 0 || lds > 160 * 1024 ||
      (mode == 2 && (size_t)S->dim * 8 <= kTMAutoBytes))
    return HYP_OK;
  const int qr = (da + kTMCols - 1) / kTMCols * kTMSeg;  // columns per region
  if (!ts.tm_part) HYP_HIP(hipMalloc(&ts.tm_part, (size_t)kTMWG * kTMPart * sizeof(double)));
  if (!ts.tm_sel) HYP_HIP(hipMalloc(&ts.tm_sel, sizeof(int)));
  TMArgs a;
  a.psi = psi;
  a.sig = sig;
  a.sel = nullptr;
  if (skip) {
    // a sparse support takes the row-batched kernel (chosen on the device)
    HYP_LAUNCH("k_tm_select", k_tm_select, dim3(1), dim3(1024), 0, st, ts.nz, db, ts.tm_sel);
    a.sel = ts.tm_sel;
    *sel = ts.tm_sel;
  }
  a.M = M;
  a.nb = S->nb;
  a.da = da;
  a.db = db;
  a.qr = qr;
  a.nch = qr / kTMSeg;
  a.astr = S->d_astr;
  a.arank = S->d_arank;
  a.bstr = S->d_bstr;
  a.brank = S->d_brank;
  a.row_nz = skip ? ts.nz : nullptr;
  a.part = ts.tm_part;
  a.fsign = pool_kind() == 0 ? 1 : 0;
  const int nwg = std::min(kTMWG, db);
  const size_t shm = (size_t)da * tsz;
  if (dt == HYP_F64) {
    HYP_HIP(hipFuncSetAttribute((const void*)k_tdens_m<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    HYP_LAUNCH("k_tdens_m", k_tdens_m<double>, dim3((unsigned)nwg), dim3(1024), shm, st, a);
  } else {
    HYP_HIP(hipFuncSetAttribute((const void*)k_tdens_m<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    HYP_LAUNCH("k_tdens_m", k_tdens_m<float>, dim3((unsigned)nwg), dim3(1024), shm, st, a);
  }
  HYP_LAUNCH("k_tm_final", k_tm_final, dim3((kBins * kBins + 2 * kBins + 255) / 256), dim3(256), 0, st, ts.tm_part,
             nwg, Ta, Tb, Tab, a.sel);
  HYP_HIP(hipGetLastError());
  *done = true;
  return HYP_OK;
}

// Transition values of singles and alpha-beta doubles (Ta, Tb, Tab) by the
// row-batched kernel.
static hyp_status tdens_rows(Sector* S, hyp_dtype dt, TScratch& ts, const void* psi, const void* sig,
                             double* Ta, double* Tb, double* Tab, bool skip, hipStream_t st, const int* sel) {
  TRArgs a;
  a.psi = psi;
  a.sig = sig;
  a.sel = sel;
  a.M = S->M;
  a.da = (int)S->da;
  a.db = (int)S->db;
  a.astr = S->d_astr;
  a.arank = S->d_arank;
  a.K = (int)binom64(S->M - 2, S->nb - 1);
  a.nsx = S->na * (S->M - S->na);
  a.Kid = a.K > 0 ? a.K : a.db;
  a.n_eb = (int)(2 * binom64(S->M, 2));
  a.n_id = (a.db + a.Kid - 1) / a.Kid;
  const int nt = std::max(64, std::min(512, (a.da + 63) / 64 * 64));
  a.nchunk = (a.da + nt - 1) / nt;
  const size_t rows_need = (size_t)a.n_eb * a.K;
  a.fsign = pool_kind() == 0 ? 1 : 0;
  if (rows_need > 0 && (ts.rows_M != S->M || ts.rows_nb != S->nb || ts.rows_fsign != a.fsign)) {
    if (rows_need > ts.rows_cap) {
      HYP_HIP(hipDeviceSynchronize());
      if (ts.rows) HYP_HIP(hipFree(ts.rows));
      ts.rows = nullptr;
      ts.rows_cap = 0;
      HYP_HIP(hipMalloc(&ts.rows, rows_need * sizeof(int2)));
      ts.rows_cap = rows_need;
    }
    HYP_LAUNCH("k_eb_rows", k_eb_rows, dim3((unsigned)((rows_need + 255) / 256)), dim3(256), 0, st, S->M, S->nb,
               a.n_eb, a.K, S->d_brank, a.fsign, ts.rows);
    ts.rows_M = S->M;
    ts.rows_nb = S->nb;
    ts.rows_fsign = a.fsign;
  }
  a.rows = ts.rows;
  a.rcount = nullptr;
  a.idrows = nullptr;
  a.n_idrows = nullptr;
  if (skip) {
    // row pairs whose source row is in psi's support (flags ts.nz, beta rows
    // first), and the identity slices over the ordered list of those rows
    if (rows_need > ts.crows_cap) {
      HYP_HIP(hipDeviceSynchronize());
      if (ts.crows) HYP_HIP(hipFree(ts.crows));
      if (ts.rcount) HYP_HIP(hipFree(ts.rcount));
      ts.crows = nullptr;
      ts.rcount = nullptr;
      ts.crows_cap = 0;
      HYP_HIP(hipMalloc(&ts.crows, rows_need * sizeof(int2)));
      HYP_HIP(hipMalloc(&ts.rcount, (size_t)a.n_eb * sizeof(int)));
      ts.crows_cap = rows_need;
    }
    if (rows_need > 0) {
      HYP_LAUNCH("k_rows_compact", k_rows_compact, dim3((unsigned)((a.n_eb + 3) / 4)), dim3(256), 0, st, ts.rows,
                 a.n_eb, a.K, ts.nz, ts.crows, ts.rcount);
      a.rows = ts.crows;
      a.rcount = ts.rcount;
    }
    a.idrows = ts.lists;
    a.n_idrows = ts.cnt;
  }
  const size_t pneed = (size_t)(a.n_eb + a.n_id) * a.nchunk * kStageW;
  if (pneed > ts.rpart_cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (ts.rpart) HYP_HIP(hipFree(ts.rpart));
    ts.rpart = nullptr;
    ts.rpart_cap = 0;
    HYP_HIP(hipMalloc(&ts.rpart, pneed * sizeof(double)));
    ts.rpart_cap = pneed;
  }
  a.part = ts.rpart;
  // the row plus a zero slot, or the flush's per-wave bins
  const size_t row_bytes = (((size_t)a.da + 1) * (dt == HYP_F64 ? 8 : 4) + 15) & ~(size_t)15;
  const size_t shm = std::max(row_bytes, (size_t)(nt / 64) * kBins * sizeof(double));
  const int64_t nslot = a.n_eb + a.n_id;
  const int64_t nblk = (int64_t)8 * ((nslot + 7) / 8) * a.nchunk;
  // compact staging: FP64 rows whose 16-byte blocks start at the row start
  if (dt == HYP_F64 && g_row_staging == 0 && nt == 512 && a.da % 2 == 0 && ((uintptr_t)psi & 15u) == 0) {
    const TScratch::CTab* ct = nullptr;
    hyp_status r = compact_tables(S, ts, nt, st, &ct);
    if (r != HYP_OK) return r;
    // LDS: buffer 0 | buffer 1 at kCBuf1 (each with its zero slot) | row pairs
    const size_t pairs_off = (size_t)kCBuf1 + ((size_t)ct->max + 1) * 16;
    const size_t cshm = std::max(pairs_off + (size_t)std::max(a.K, a.Kid) * sizeof(int2),
                                 (size_t)(nt / 64) * kBins * sizeof(double));
    if (ct->ok && cshm <= 160 * 1024 - 256) {
      HYP_HIP(hipFuncSetAttribute((const void*)k_tdens_rows_c, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)cshm));
      HYP_LAUNCH("k_tdens_rows", k_tdens_rows_c, dim3((unsigned)nblk), dim3(nt), cshm, st, a, ct->bpos, ct->blist,
                 ct->nb, (a.da + 1) / 2, (uint32_t)pairs_off);
      HYP_LAUNCH("k_tdens_rows_final", k_tdens_rows_final, dim3((kBins * kStageW + kBins + 255) / 256), dim3(256),
                 0, st, ts.rpart, a.n_eb, a.n_id, a.nchunk, Ta, Tb, Tab, sel);
      return HYP_OK;
    }
  }
  if (dt == HYP_F64) {
    if (shm > 48 * 1024)
      HYP_HIP(hipFuncSetAttribute((const void*)k_tdens_rows<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm));
    HYP_LAUNCH("k_tdens_rows", k_tdens_rows<double>, dim3((unsigned)nblk), dim3(nt), shm, st, a);
  } else {
    if (shm > 48 * 1024)
      HYP_HIP(hipFuncSetAttribute((const void*)k_tdens_rows<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm));
    HYP_LAUNCH("k_tdens_rows", k_tdens_rows<float>, dim3((unsigned)nblk), dim3(nt), shm, st, a);
  }
  HYP_LAUNCH("k_tdens_rows_final", k_tdens_rows_final, dim3((kBins * kStageW + kBins + 255) / 256), dim3(256), 0,
             st, ts.rpart, a.n_eb, a.n_id, a.nchunk, Ta, Tb, Tab, sel);
  return HYP_OK;
}

// Row and column support flags of psi ([db] beta rows, then [da] alpha
// columns) in this device's sweep scratch, valid until the next call on the
// device; also sizes the support lists and their counters.
hyp_status support_flags(Sector* S, hyp_dtype dt, const void* psi, const uint32_t** flags, hipStream_t st) {
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  TScratch& ts = g_ts[dev];
  const int64_t da = S->da, db = S->db;
  const size_t nneed = (size_t)(da + db);
  if (nneed > ts.nz_cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (ts.nz) HYP_HIP(hipFree(ts.nz));
    if (ts.lists) HYP_HIP(hipFree(ts.lists));
    ts.nz = nullptr;
    ts.lists = nullptr;
    ts.nz_cap = 0;
    HYP_HIP(hipMalloc(&ts.nz, nneed * sizeof(uint32_t)));
    HYP_HIP(hipMalloc(&ts.lists, nneed * sizeof(int)));
    ts.nz_cap = nneed;
  }
  if (!ts.cnt) {
    HYP_HIP(hipMalloc(&ts.cnt, 2 * sizeof(int)));
  }
  HYP_LAUNCH("k_zero_u32", k_zero_u32, dim3((unsigned)std::min<int64_t>(1024, (da + db + 255) / 256)), dim3(256), 0,
             st, ts.nz, (int)(da + db));
  dim3 tg((unsigned)((da + 63) / 64), (unsigned)((db + 63) / 64));
  if (dt == HYP_F64)
    HYP_LAUNCH("k_support", k_support<double>, tg, dim3(256), 0, st, (const double*)psi, (int)db, (int)da, ts.nz,
               ts.nz + db);
  else
    HYP_LAUNCH("k_support", k_support<float>, tg, dim3(256), 0, st, (const float*)psi, (int)db, (int)da, ts.nz,
               ts.nz + db);
  *flags = ts.nz;
  return HYP_OK;
}

hyp_status launch_tdens(Sector* S, hyp_dtype dt, const hyp_exc* ops, int64_t n_ops, const void* psi,
                        const void* sig, double* grad, hipStream_t st, bool bins) {
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  TScratch& ts = g_ts[dev];
  if (!ts.binom) {
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
    HYP_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom_s), tab, sizeof(tab)));
    HYP_HIP(hipMalloc(&ts.T, sizeof(double) * (2 * kBins + kBins * kBins)));
    HYP_HIP(hipMalloc(&ts.red, sizeof(double) * ((size_t)kBins * kRowSlices * kStageW + (size_t)kRowBlocks * kBins)));
    ts.binom = true;
  }
  double* Ta = ts.T;
  double* Tb = ts.T + kBins;
  double* Tab = ts.T + 2 * kBins;
  const int64_t da = S->da, db = S->db;
  // support skipping: only amplitudes in psi's support enter T(tau) = sum_D
  // s sigma[tau D] psi[D], so the row pairs and Gram sums are restricted to
  // psi's nonzero beta rows and alpha columns
  const bool skip = support_skip() && !bins;
  if (skip) {
    const uint32_t* nz = nullptr;
    hyp_status rs = support_flags(S, dt, psi, &nz, st);
    if (rs != HYP_OK) return rs;
    HYP_LAUNCH("k_list_nz", k_list_nz, dim3(1), dim3(1024), 0, st, ts.nz, (int)db, ts.lists, ts.cnt);
    HYP_LAUNCH("k_list_nz", k_list_nz, dim3(1), dim3(1024), 0, st, ts.nz + db, (int)da, ts.lists + db, ts.cnt + 1);
  }
  if (!bins) {
    bool done = false;
    const int* sel = nullptr;
    hyp_status r = tdens_mm(S, dt, ts, psi, sig, Ta, Tb, Tab, skip, st, &done, &sel);
    // with a device-side choice both forms are launched; the other exits at once
    if (r == HYP_OK && (!done || sel)) r = tdens_rows(S, dt, ts, psi, sig, Ta, Tb, Tab, skip, st, sel);
    if (r != HYP_OK) return r;
  } else {
  const size_t need = tdens_bytes(S);
  if (need > ts.cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (ts.part) HYP_HIP(hipFree(ts.part));
    ts.part = nullptr;
    ts.cap = 0;
    HYP_HIP(hipMalloc(&ts.part, need));
    ts.cap = need;
  }
  TArgs a;
  a.psi = psi;
  a.sig = sig;
  a.M = S->M;
  a.nb = S->nb;
  a.da = (int)S->da;
  a.db = (int)S->db;
  a.astr = S->d_astr;
  a.bstr = S->d_bstr;
  a.arank = S->d_arank;
  a.brank = S->d_brank;
  const int nt = std::max(64, std::min(768, (a.da + 63) / 64 * 64));
  a.nchunk = (a.da + nt - 1) / nt;
  a.nstage = 1 + a.nb * (a.M - a.nb);
  a.part = ts.part;
  a.fsign = pool_kind() == 0 ? 1 : 0;
  const size_t shm = (size_t)a.da * (dt == HYP_F64 ? 8 : 4);
  const int64_t nblk = (int64_t)8 * ((a.db + 7) / 8) * a.nchunk;
  if (dt == HYP_F64) {
    if (shm > 48 * 1024)
      HYP_HIP(hipFuncSetAttribute((const void*)k_tdens<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    HYP_LAUNCH("k_tdens", k_tdens<double>, dim3((unsigned)nblk), dim3(nt), shm, st, a);
  } else {
    if (shm > 48 * 1024)
      HYP_HIP(hipFuncSetAttribute((const void*)k_tdens<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    HYP_LAUNCH("k_tdens", k_tdens<float>, dim3((unsigned)nblk), dim3(nt), shm, st, a);
  }
  double* red_ab = ts.red;
  double* red_a = ts.red + (size_t)kBins * kRowSlices * kStageW;
  HYP_LAUNCH("k_tdens_reduce_ab", k_tdens_reduce_ab, dim3(kBins, kRowSlices), dim3(256), 0, st, a, red_ab);
  HYP_LAUNCH("k_tdens_reduce_a", k_tdens_reduce_a, dim3(kRowBlocks), dim3(256), 0, st, a, red_a);
  HYP_LAUNCH("k_tdens_final", k_tdens_final, dim3((kBins * kStageW + kBins + 255) / 256), dim3(256), 0, st,
             red_ab, red_a, Ta, Tb, Tab);
  }
  // same-spin doubles: per-core Gram blocks of both string spaces (only the
  // string pairs one same-spin double apart), then the gather
  const size_t na_g = core_gram_doubles(S->M, S->na), nb_g = core_gram_doubles(S->M, S->nb);
  const size_t wneed = 2 * (size_t)std::max(da * ((db + 1) & ~(int64_t)1), db * ((da + 1) & ~(int64_t)1));
  const size_t gneed = na_g + nb_g + ((na_g + nb_g) > 0 ? wneed : 0);
  if (gneed > ts.gram_cap) {
    HYP_HIP(hipDeviceSynchronize());
    if (ts.gram) HYP_HIP(hipFree(ts.gram));
    ts.gram = nullptr;
    ts.gram_cap = 0;
    HYP_HIP(hipMalloc(&ts.gram, gneed * sizeof(double)));
    ts.gram_cap = gneed;
  }
  double* Ga = ts.gram;
  double* Gb = Ga + na_g;
  double* work = Gb + nb_g;
  if (na_g > 0) {
    // alpha strings as rows, beta rows as columns: element (alpha I, beta k)
    // of the [beta][alpha] state at I + k * D_a
    CoreGramCall g{"k_core_gram_a", S->M, S->na, &S->h_arank, dt == HYP_F64, psi, sig, 1, da, (int)da, (int)db,
                   skip ? ts.lists : nullptr, skip ? ts.cnt : nullptr, skip ? ts.nz + db : nullptr, work, Ga};
    hyp_status r = launch_core_gram(g, st);
    if (r != HYP_OK) return r;
  }
  if (nb_g > 0) {
    CoreGramCall g{"k_core_gram_b", S->M, S->nb, &S->h_brank, dt == HYP_F64, psi, sig, da, 1, (int)db, (int)da,
                   skip ? ts.lists + db : nullptr, skip ? ts.cnt + 1 : nullptr, skip ? ts.nz : nullptr, work, Gb};
    hyp_status r = launch_core_gram(g, st);
    if (r != HYP_OK) return r;
  }
  const CoreSpace csa = core_space(S->M, S->na), csb = core_space(S->M, S->nb);
  HYP_LAUNCH("k_gram_grad", k_gram_grad, dim3((unsigned)n_ops), dim3(256), 0, st, ops, S->M, S->na, S->nb, Ga,
             csa.S, Gb, csb.S, pool_kind() == 0 ? 1 : 0, grad);
  int* rec = bad_exc_record();
  if (!rec) return fail(HYP_ERR_HIP, "excitation check record not found");
  HYP_LAUNCH("k_tdens_grad", k_tdens_grad, dim3((unsigned)((n_ops + 255) / 256)), dim3(256), 0, st, ops, n_ops,
             S->M, Ta, Tb, Tab, grad, rec);
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

}  // namespace hyp

extern "C" hyp_status hyp_set_row_staging(int mode) {
  if (mode != 0 && mode != 1) return hyp::fail(HYP_ERR_ARG, "hyp_set_row_staging: mode must be 0 or 1");
  hyp::g_row_staging = mode;
  return HYP_OK;
}
