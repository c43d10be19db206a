// Same-spin doubles of the pool-gradient sweep as per-core Gram blocks.
//
// A same-spin double tau = a+_{c1} a+_{c2} a_{a2} a_{a1} pairs each string J
// that holds a1, a2 and not c1, c2 with I = J - {a1, a2} + {c1, c2}; its
// gradient needs, per pair, the sum over the other spin's strings k of
//   sigma(I, k) psi(J, k) - sigma(J, k) psi(I, k)
// (g = 2 <sigma|A psi>, the ADAPT selection quantity of the paper's
// "Numerical performance" section).  I and J share the (N-2)-electron core
// K = I & J.  The strings that contain a core K are K plus one of the C(F, 2)
// pairs of the F = M - N + 2 orbitals outside K (the core's slots), and every
// same-spin double-excitation pair of the string space is a pair of disjoint
// slots of exactly one core.  The sampled Gram the gradients need is therefore
// a set of small dense Grams, one S x S block per core (S = C(F, 2): 45 at 16
// orbitals and 8 electrons, 8,008 cores), each a contraction over the K
// columns of the slots' rows:
//   Gc[core][i][j] = sum_k X[s_i][k] Y[s_j][k]     X = sigma rows, Y = psi rows
// 62% of a block's entries are disjoint-slot pairs that a generator reads,
// against 6% of the full string-space Gram.
//
// Kernel: one workgroup of 256 threads (4 waves) per (core, 48 x 48 tile of
// the block).  Each wave holds the whole tile as 3 x 3 FP64 MFMA blocks
// (v_mfma_f64_16x16x4_f64: per 4 columns one 8-byte operand per lane for
// each 16-slot row block of X and of Y) over its quarter of every 32-column
// chunk, and the four waves add their tiles in LDS at the end.  Chunks of
// the 96 rows are staged by direct global->LDS copies into two alternating
// buffers, the next copy in flight while the current one is multiplied;
// rows are padded to 34 doubles.  A dense contraction, so the matrix cores:
// the same FP64 peak as the vector ALU on this chip, but a third of the
// registers of a 6 x 6 per-lane register tile, hence more resident waves to
// cover the copies, and 6 LDS reads per 9 MFMAs.
#include "hyp_internal.h"

#include <algorithm>
#include <vector>

namespace hyp {

constexpr int kGT = 48;                            // tile edge in slots (8 lanes x 6)
constexpr int kGC = 32;                            // columns per staged chunk
constexpr int kGLd = kGC + 2;                      // LDS row stride in doubles
constexpr int kGRows = 2 * kGT;                    // X rows, then Y rows
constexpr int kGPieces = kGRows * (kGLd / 2);      // 16-byte LDS pieces per buffer
constexpr uint32_t kGBufBytes = kGPieces * 16u;    // 26,112
constexpr int kGThreads = 256;
constexpr int kGPer = (kGPieces + kGThreads - 1) / kGThreads;
constexpr uint32_t kGLdsBytes = 2 * kGBufBytes + kGRows * 4 + 16;
typedef double f64x2 __attribute__((ext_vector_type(2)));  // one 16-byte LDS read or write
typedef double f64x4 __attribute__((ext_vector_type(4)));  // a lane's part of a 16 x 16 MFMA block

struct GramArgs {
  const double* X;        // dense FP64 rows (sigma), row r at X + r * ld
  const double* Y;        // (psi)
  int64_t ld;
  int dma;                // 1: X, Y 16-byte aligned and ld even (direct copies)
  const void* Xs;         // storage-type operands of the gathered path:
  const void* Ys;         //   element (row r, column k) at [r * rs + k * cs]
  int64_t rs, cs;
  int K;                  // columns
  const int* klist;       // support skipping: psi's nonzero columns and their
  const int* kcount;      //   number; gathered columns when 2 * count <= K
  const uint32_t* rflag;  // support skipping: psi's nonzero rows (a tile none reaches is zero)
  const int* rows;        // [ncore][S] string rank of every slot
  int S, ntile;
  int64_t nwork;          // ncore * ntile^2
  int64_t per_xcd;        // ceil(nwork / 8)
  double* G;              // [ncore][S][S]
};

__device__ inline bool gram_gathered(const GramArgs& a) { return a.klist && 2 * (*a.kcount) <= a.K; }

template <typename T>
__global__ void __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(3))) k_core_gram(GramArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* s_row = (int*)(smem + 2 * kGBufBytes);
  int* s_any = s_row + kGRows;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // cores in colex order share strings: consecutive items go to one XCD
  const int64_t b = blockIdx.x;
  const int64_t item = (b & 7) * a.per_xcd + (b >> 3);
  if (item >= a.nwork) return;
  const int nt2 = a.ntile * a.ntile;
  const int64_t core = item / nt2;
  const int t = (int)(item - core * nt2);
  const int ti = t / a.ntile, tj = t - ti * a.ntile;
  if (tid < kGRows) {
    const int slot = tid < kGT ? ti * kGT + tid : tj * kGT + tid - kGT;
    const int rr = slot < a.S ? a.rows[core * a.S + slot] : -1;
    s_row[tid] = rr;
  }
  if (tid == 0) *s_any = a.rflag ? 0 : 1;
  __syncthreads();
  if (a.rflag && tid >= kGT && tid < kGRows && s_row[tid] >= 0 && a.rflag[s_row[tid]] != 0u) *s_any = 1;
  __syncthreads();
  double* Gt = a.G + core * a.S * a.S;
  if (!*s_any) {
    // no psi row of the tile's Y slots is nonzero: the tile is zero
    for (int e = tid; e < kGT * kGT; e += kGThreads) {
      const int gi = ti * kGT + e / kGT, gj = tj * kGT + e % kGT;
      if (gi < a.S && gj < a.S) Gt[(int64_t)gi * a.S + gj] = 0.0;
    }
    return;
  }
  // this thread's pieces of a buffer: LDS piece q = j * 256 + tid holds
  // columns 2 col, 2 col + 1 of staged row q / 17 (col = q % 17; col 16
  // pads), rows below kGT from X, the others from Y; off[j] = the piece's
  // first element in its operand (row * ld + 2 col), -1 for no piece (a pad
  // column or a row without a slot)
  int off[kGPer];
#pragma unroll
  for (int j = 0; j < kGPer; ++j) {
    const int q = j * kGThreads + tid;
    const int row = q / (kGLd / 2), col = q - row * (kGLd / 2);
    const bool act = q < kGPieces && col < kGC / 2 && s_row[row] >= 0;
    off[j] = act ? (int)((int64_t)s_row[row] * a.ld + 2 * col) : -1;
  }
  const uint32_t buf0 = lds_addr(smem), buf1 = buf0 + kGBufBytes;
  // MFMA operands: lane l supplies row (l & 15) of a 16-slot block at column
  // (l >> 4) of each 4-column step; block (bi, bj) of the result holds
  // Gc[16 bi + (l >> 4) + 4 e][16 bj + (l & 15)] in element e of lane l
  const int mr = lane & 15, mk = lane >> 4;
  f64x4 acc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  auto compute = [&](uint32_t buf) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const uint32_t kb = (uint32_t)(8 * w + 4 * s + mk) * 8u;
      double x[3], y[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        x[i] = lds_load<double>(buf + (uint32_t)((16 * i + mr) * kGLd) * 8u + kb);
        y[i] = lds_load<double>(buf + (uint32_t)((kGT + 16 * i + mr) * kGLd) * 8u + kb);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[i], y[j], acc[i][j], 0, 0, 0);
    }
  };
  // columns [k0, k0 + kn) through registers, zeros past kn and on rows
  // without a slot; gathered columns when kl is given
  auto stage_regs = [&](uint32_t buf, int k0, int kn, const int* kl) {
#pragma unroll
    for (int j = 0; j < kGPer; ++j) {
      const int q = j * kGThreads + tid;
      const int row = q / (kGLd / 2), col = q - row * (kGLd / 2);
      if (q < kGPieces && col < kGC / 2) {
        double v0 = 0.0, v1 = 0.0;
        const int64_t rr = s_row[row];
        if (rr >= 0) {
          const int k = 2 * col;
          if (kl) {
            const T* base = (const T*)(row < kGT ? a.Xs : a.Ys);
            if (k < kn) v0 = (double)base[rr * a.rs + (int64_t)kl[k0 + k] * a.cs];
            if (k + 1 < kn) v1 = (double)base[rr * a.rs + (int64_t)kl[k0 + k + 1] * a.cs];
          } else {
            const double* src = (row < kGT ? a.X : a.Y) + rr * a.ld + k0;
            if (k < kn) v0 = src[k];
            if (k + 1 < kn) v1 = src[k + 1];
          }
        }
        f64x2 v;
        v.x = v0;
        v.y = v1;
        *(__attribute__((address_space(3))) f64x2*)(uintptr_t)(buf + (uint32_t)q * 16u) = v;
      }
    }
  };
  if (gram_gathered(a)) {
    const int kc = *a.kcount;
    for (int k0 = 0; k0 < kc; k0 += kGC) {
      stage_regs(buf0, k0, min(kGC, kc - k0), a.klist);
      __syncthreads();
      compute(buf0);
      __syncthreads();
    }
  } else {
    const int nfull = a.dma ? a.K / kGC : 0;
    auto issue = [&](uint32_t buf, int k0) {
#pragma unroll
      for (int j = 0; j < kGPer; ++j) {
        const int base = j * kGThreads + w * 64;  // wave-uniform first piece
        if (base < kGPieces) {
          const uint32_t dst = (uint32_t)__builtin_amdgcn_readfirstlane(buf + (uint32_t)base * 16u);
          // pieces of rows below kGT come from X (base + lane below 17 kGT)
          const double* op = (j * kGThreads + tid) < kGT * (kGLd / 2) ? a.X : a.Y;
          if (off[j] >= 0) dma16(dst, op + off[j] + k0);
        }
      }
    };
    if (nfull > 0) {
      // rows without a slot stay unwritten in the direct copies: clear them
      // once in both buffers (only the dropped tile entries read them)
      stage_regs(buf0, 0, 0, nullptr);
      stage_regs(buf1, 0, 0, nullptr);
      __syncthreads();
      issue(buf0, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    for (int ch = 0; ch < nfull; ++ch) {
      const uint32_t cur = (ch & 1) ? buf1 : buf0, nxt = (ch & 1) ? buf0 : buf1;
      if (ch + 1 < nfull) issue(nxt, (ch + 1) * kGC);
      compute(cur);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();  // chunk ch + 1 copied by every wave; chunk ch's reads done
    }
    // the ragged tail (or every chunk without direct copies)
    for (int k0 = nfull * kGC; k0 < a.K; k0 += kGC) {
      stage_regs(buf0, k0, min(kGC, a.K - k0), nullptr);
      __syncthreads();
      compute(buf0);
      __syncthreads();
    }
  }
  // the four waves' tiles summed in LDS in a fixed order; wave 3 stores
  double* red = (double*)smem;
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int li = 16 * i + mk + 4 * e, lj = 16 * j + mr;
            double v = acc[i][j][e];
            if (ww > 0) v += red[li * kGT + lj];
            if (ww < 3) {
              red[li * kGT + lj] = v;
            } else {
              const int gi = ti * kGT + li, gj = tj * kGT + lj;
              if (gi < a.S && gj < a.S) Gt[(int64_t)gi * a.S + gj] = v;
            }
          }
    }
    __syncthreads();
  }
}

// Dense FP64 operand rows of a core Gram: out[c][r] = in[r][c] (transpose)
// with row stride ldo; not run when the Gram takes gathered columns.
template <typename T>
__global__ void __launch_bounds__(256) k_gram_transpose(const T* __restrict__ in, double* __restrict__ out, int rows,
                                                        int cols, int64_t ldo, const int* kcount, int K) {
  if (kcount && 2 * (*kcount) <= K) return;
  __shared__ double tile[64][65];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int rr = ty; rr < 64; rr += 4) {
    const int gr = r0 + rr, gc = c0 + tx;
    if (gr < rows && gc < cols) tile[rr][tx] = (double)in[(int64_t)gr * cols + gc];
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int gc = c0 + cc, gr = r0 + tx;
    if (gr < rows && gc < cols) out[(int64_t)gc * ldo + gr] = tile[tx][cc];
  }
}

// out[r][c] = in[r][c] widened to FP64, row stride ldo; not run when the
// Gram takes gathered columns.
template <typename T>
__global__ void __launch_bounds__(256) k_gram_widen(const T* __restrict__ in, double* __restrict__ out, int rows,
                                                    int cols, int64_t ldo, const int* kcount, int K) {
  if (kcount && 2 * (*kcount) <= K) return;
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rr = i / cols, cc = i - rr * cols;
    out[rr * ldo + cc] = (double)in[i];
  }
}

namespace {
// Slot tables of a string space, one per (orbitals, electrons) seen on the
// device, oldest replaced first.
struct SlotTab {
  int M = -1, N = -1, ncore = 0, S = 0;
  int* rows = nullptr;
};
struct CoreCache {
  SlotTab tab[8];
  int next = 0;
};
CoreCache g_cc[64];

int64_t nck(int m, int k) {
  if (k < 0 || m < 0 || k > m) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (m - k + i) / i;
  return r;
}
}  // namespace

CoreSpace core_space(int M, int N) {
  CoreSpace cs;
  if (N < 2 || M - N < 2) return cs;  // no same-spin double
  cs.F = M - N + 2;
  cs.S = (int)nck(cs.F, 2);
  cs.ncore = nck(M, N - 2);
  cs.ntile = (cs.S + kGT - 1) / kGT;
  return cs;
}

// Host tables of the string space (M, N): rows[core][slot] = rank of the
// string core | p | q, cores in colex order (increasing masks), slot
// w (w - 1) / 2 + u for the u-th < w-th orbital outside the core, and
// masks[core] = the core's orbitals.
hyp_status core_tables_host(int M, int N, const RankTables& R, std::vector<int>& rows,
                            std::vector<uint32_t>& masks) {
  const CoreSpace cs = core_space(M, N);
  try {
    rows.assign((size_t)cs.ncore * cs.S, 0);
    masks.assign((size_t)cs.ncore, 0u);
  } catch (...) {
    return fail(HYP_ERR_NOMEM, "core tables: host allocation failed");
  }
  const uint32_t full = (1u << M) - 1u;
  const int k = N - 2;
  uint32_t core = (k == 0) ? 0u : ((1u << k) - 1u);
  for (int64_t ci = 0; ci < cs.ncore; ++ci) {
    masks[(size_t)ci] = core;
    int comp[16];
    int nf = 0;
    for (int o = 0; o < M; ++o)
      if (!(core >> o & 1u)) comp[nf++] = o;
    for (int wv = 1; wv < nf; ++wv)
      for (int u = 0; u < wv; ++u) {
        const uint32_t s = core | (1u << comp[u]) | (1u << comp[wv]);
        rows[(size_t)ci * cs.S + wv * (wv - 1) / 2 + u] = R.lo[s & 255u] + R.hi[(s >> 8) & 255u];
      }
    if (k > 0) {  // next mask with k bits (Gosper)
      const uint32_t lo = core & (~core + 1u), rip = core + lo;
      core = (((rip ^ core) >> 2) / lo) | rip;
      if (ci + 1 < cs.ncore && (core & ~full)) return fail(HYP_ERR_HIP, "core enumeration overflow");
    }
  }
  return HYP_OK;
}

// Device copy of the slot table of (M, N), cached per device.
static hyp_status slot_rows(int M, int N, const RankTables& R, const int** out) {
  int dev = 0;
  HYP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(HYP_ERR_HIP, "device index out of range");
  CoreCache& cc = g_cc[dev];
  for (const SlotTab& t : cc.tab)
    if (t.M == M && t.N == N) {
      *out = t.rows;
      return HYP_OK;
    }
  const CoreSpace cs = core_space(M, N);
  std::vector<int> h;
  std::vector<uint32_t> hm;
  hyp_status rt = core_tables_host(M, N, R, h, hm);
  if (rt != HYP_OK) return rt;
  SlotTab& t = cc.tab[cc.next];
  if (t.rows) {
    HYP_HIP(hipDeviceSynchronize());  // queued launches may still read the replaced table
    HYP_HIP(hipFree(t.rows));
  }
  t = SlotTab();
  HYP_HIP(hipMalloc(&t.rows, std::max<size_t>(1, h.size()) * sizeof(int)));
  HYP_HIP(hipMemcpy(t.rows, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
  t.M = M;
  t.N = N;
  t.ncore = (int)cs.ncore;
  t.S = cs.S;
  cc.next = (cc.next + 1) % 8;
  *out = t.rows;
  return HYP_OK;
}

hyp_status launch_core_gram(const CoreGramCall& g, hipStream_t st) {
  const CoreSpace cs = core_space(g.M, g.N);
  if (cs.ncore == 0) return HYP_OK;
  const int* rows = nullptr;
  hyp_status rs = slot_rows(g.M, g.N, *g.rank_host, &rows);
  if (rs != HYP_OK) return rs;
  const int64_t ld = ((int64_t)g.K + 1) & ~(int64_t)1;
  GramArgs a;
  a.rs = g.rs;
  a.cs = g.cs;
  a.Xs = g.sig;
  a.Ys = g.psi;
  a.K = g.K;
  a.klist = g.klist;
  a.kcount = g.kcount;
  a.rflag = g.rflag;
  a.rows = rows;
  a.S = cs.S;
  a.ntile = cs.ntile;
  a.nwork = cs.ncore * (int64_t)cs.ntile * cs.ntile;
  a.per_xcd = (a.nwork + 7) / 8;
  a.G = g.G;
  // dense FP64 operand rows: the storage itself when its rows already are
  // (FP64, rows along the columns, 16-byte aligned, even length), else
  // copies (transposed and/or widened) into the work area with even stride
  const bool direct = g.f64 && g.cs == 1 && g.rs == g.K && (g.K % 2 == 0) &&
                      ((uintptr_t)g.psi & 15u) == 0 && ((uintptr_t)g.sig & 15u) == 0;
  if (direct) {
    a.X = (const double*)g.sig;
    a.Y = (const double*)g.psi;
    a.ld = g.K;
  } else {
    double* xw = g.work;
    double* yw = g.work + (int64_t)g.nrow * ld;
    if (g.cs == 1) {  // rows along the columns already: widen (or re-stride)
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, ((int64_t)g.nrow * g.K + 255) / 256));
      if (g.f64) {
        HYP_LAUNCH("k_gram_widen", k_gram_widen<double>, dim3(grid), dim3(256), 0, st, (const double*)g.sig, xw,
                   g.nrow, g.K, ld, g.kcount, g.K);
        HYP_LAUNCH("k_gram_widen", k_gram_widen<double>, dim3(grid), dim3(256), 0, st, (const double*)g.psi, yw,
                   g.nrow, g.K, ld, g.kcount, g.K);
      } else {
        HYP_LAUNCH("k_gram_widen", k_gram_widen<float>, dim3(grid), dim3(256), 0, st, (const float*)g.sig, xw,
                   g.nrow, g.K, ld, g.kcount, g.K);
        HYP_LAUNCH("k_gram_widen", k_gram_widen<float>, dim3(grid), dim3(256), 0, st, (const float*)g.psi, yw,
                   g.nrow, g.K, ld, g.kcount, g.K);
      }
    } else {  // storage [K][nrow]: transpose
      const dim3 tg((unsigned)((g.nrow + 63) / 64), (unsigned)((g.K + 63) / 64));
      if (g.f64) {
        HYP_LAUNCH("k_gram_transpose", k_gram_transpose<double>, tg, dim3(256), 0, st, (const double*)g.sig, xw, g.K,
                   g.nrow, ld, g.kcount, g.K);
        HYP_LAUNCH("k_gram_transpose", k_gram_transpose<double>, tg, dim3(256), 0, st, (const double*)g.psi, yw, g.K,
                   g.nrow, ld, g.kcount, g.K);
      } else {
        HYP_LAUNCH("k_gram_transpose", k_gram_transpose<float>, tg, dim3(256), 0, st, (const float*)g.sig, xw, g.K,
                   g.nrow, ld, g.kcount, g.K);
        HYP_LAUNCH("k_gram_transpose", k_gram_transpose<float>, tg, dim3(256), 0, st, (const float*)g.psi, yw, g.K,
                   g.nrow, ld, g.kcount, g.K);
      }
    }
    a.X = xw;
    a.Y = yw;
    a.ld = ld;
  }
  a.dma = (a.ld % 2 == 0) && (((uintptr_t)a.X | (uintptr_t)a.Y) & 15u) == 0;
  const unsigned grid = (unsigned)(8 * a.per_xcd);
  if (g.f64) {
    HYP_HIP(hipFuncSetAttribute((const void*)k_core_gram<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kGLdsBytes));
    HYP_LAUNCH(g.name, k_core_gram<double>, dim3(grid), dim3(kGThreads), kGLdsBytes, st, a);
  } else {
    HYP_HIP(hipFuncSetAttribute((const void*)k_core_gram<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kGLdsBytes));
    HYP_LAUNCH(g.name, k_core_gram<float>, dim3(grid), dim3(kGThreads), kGLdsBytes, st, a);
  }
  HYP_HIP(hipGetLastError());
  return HYP_OK;
}

size_t core_gram_doubles(int M, int N) {
  const CoreSpace cs = core_space(M, N);
  return (size_t)cs.ncore * cs.S * cs.S;
}

}  // namespace hyp
