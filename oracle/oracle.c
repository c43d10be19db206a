/*
 * Plain FP64 CPU oracle for the sparse state-vector ADAPT-VQE path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU
 * library is checked against.  It shares no code, header or table with the
 * GPU library and is never linked into it.  Everything here is the literal
 * definition of the operation, term by term or pair by pair, with no
 * grouping, compression, blocking or reordering.
 *
 * Conventions (the same data model the GPU side implements separately):
 *   n = 2M qubits, qubit q < M = orbital q spin alpha, q >= M = orbital q-M
 *   spin beta; bit set = occupied.  A sector (N_a, N_b) state is addressed
 *   by idx(b) = rank(beta) * C(M, N_a) + rank(alpha), with the colex rank
 *   rank_k(s) = sum_{i=1..k} C(o_i, i) over the set bits o_1 < ... < o_k.
 *   This is the position of b among all sector bitstrings sorted
 *   ascending, i.e. the symmetry-restricted configuration space Omega_CIk
 *   of the paper ("Sparse State-Vector Emulation", Table 1).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------------------------------------------------------- binomials */

static int64_t binom_tab[65][65];

#include <omp.h>
/* thread count of the parallel loops below (timing at 1 thread and at all) */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }

__attribute__((constructor)) static void binom_init(void) {
    /* Pascal's triangle */
    for (int m = 0; m <= 64; ++m) {
        binom_tab[m][0] = 1;
        for (int k = 1; k <= m; ++k)
            binom_tab[m][k] = binom_tab[m - 1][k - 1] + (k <= m - 1 ? binom_tab[m - 1][k] : 0);
    }
}

static int64_t orc_choose(int m, int k) {
    if (k < 0 || m < 0 || k > m) return 0;
    return binom_tab[m][k];
}

static int popc32(uint32_t v) { return __builtin_popcount(v); }

int64_t orc_binom(int m, int k) { return orc_choose(m, k); }

/* colex rank of a k-subset given as a bitmask */
int64_t orc_rank_string(uint32_t s) {
    int64_t r = 0;
    int i = 0;
    for (int o = 0; o < 32; ++o) {
        if (s & (1u << o)) {
            ++i;
            r += orc_choose(o, i);
        }
    }
    return r;
}

/* inverse of orc_rank_string: the k-subset of {0..m-1} with the given rank */
uint32_t orc_unrank_string(int m, int k, int64_t r) {
    uint32_t s = 0;
    for (int i = k; i >= 1; --i) {
        int o = i - 1;
        while (o + 1 < m && orc_choose(o + 1, i) <= r) ++o;
        r -= orc_choose(o, i);
        s |= 1u << o;
    }
    return s;
}

typedef struct {
    int M, na, nb;
    int64_t da, db, dim;
    uint32_t amask;
} sector_t;

static void sector_init(sector_t *S, int M, int na, int nb) {
    S->M = M; S->na = na; S->nb = nb;
    S->da = orc_choose(M, na);
    S->db = orc_choose(M, nb);
    S->dim = S->da * S->db;
    S->amask = (M >= 32) ? 0xffffffffu : ((1u << M) - 1u);
}

static int in_sector(const sector_t *S, uint32_t b) {
    return popc32(b & S->amask) == S->na && popc32(b >> S->M) == S->nb;
}

static int64_t sector_rank(const sector_t *S, uint32_t b) {
    return orc_rank_string(b >> S->M) * S->da + orc_rank_string(b & S->amask);
}

static uint32_t sector_unrank(const sector_t *S, int64_t idx) {
    int64_t rb = idx / S->da, ra = idx % S->da;
    return orc_unrank_string(S->M, S->na, ra) | (orc_unrank_string(S->M, S->nb, rb) << S->M);
}

int64_t orc_sector_dim(int M, int na, int nb) {
    sector_t S; sector_init(&S, M, na, nb); return S.dim;
}

void orc_sector_rank(int M, int na, int nb, const uint32_t *bits, int64_t n, int64_t *idx) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int64_t i = 0; i < n; ++i) idx[i] = in_sector(&S, bits[i]) ? sector_rank(&S, bits[i]) : -1;
}

void orc_sector_unrank(int M, int na, int nb, const int64_t *idx, int64_t n, uint32_t *bits) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int64_t i = 0; i < n; ++i) bits[i] = sector_unrank(&S, idx[i]);
}

/* -------------------------------------------------------------- H times psi */

/*
 * sigma[d] = sum_t c_t <d| P_t |b> psi[b],  b = d xor x_t,
 * with P(x,z)|b> = i^{n_Y} (-1)^{popc(z & b)} |b xor x>, n_Y = popc(x & z).
 * The paper's Hamiltonian is real (time-reversal symmetric molecules,
 * "General Framework for Variational Algorithms"), so a real coefficient
 * needs even n_Y and i^{n_Y} = (-1)^{n_Y/2}; an odd n_Y returns -1.
 * Terms whose source b falls outside the sector are skipped (P_S H P_S).
 * Outputs: the n_out sector indices out_idx[] (or all of [0, dim) if
 * out_idx == NULL, then n_out must equal dim).
 */
int orc_apply_h(int M, int na, int nb, int64_t nterm, const uint32_t *x, const uint32_t *z,
                const double *c, const double *psi, const int64_t *out_idx, int64_t n_out,
                double *out) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int64_t t = 0; t < nterm; ++t)
        if (popc32(x[t] & z[t]) & 1) return -1;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_out; ++i) {
        int64_t d = out_idx ? out_idx[i] : i;
        uint32_t bd = sector_unrank(&S, d);
        double acc = 0.0;
        for (int64_t t = 0; t < nterm; ++t) {
            uint32_t b = bd ^ x[t];
            if (!in_sector(&S, b)) continue;
            int ny = popc32(x[t] & z[t]);
            double ph = ((ny / 2) & 1) ? -1.0 : 1.0;
            if (popc32(z[t] & b) & 1) ph = -ph;
            acc += c[t] * ph * psi[sector_rank(&S, b)];
        }
        out[i] = acc;
    }
    return 0;
}

/*
 * sigma = H psi for a psi given by its nonzeros (sector indices, values):
 * every term applied to every nonzero basis state b, adding
 * c_t (-1)^{n_Y/2} (-1)^{popc(z_t & b)} psi[b] to sigma[b ^ x_t] when that
 * state is in the sector (the definition of orc_apply_h summed from the input
 * side).  out holds all dim entries and is overwritten.  -1 on an odd-n_Y term.
 */
int orc_apply_h_sparse(int M, int na, int nb, int64_t nterm, const uint32_t *x, const uint32_t *z,
                       const double *c, int64_t n_in, const int64_t *in_idx, const double *in_val,
                       double *out) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int64_t t = 0; t < nterm; ++t)
        if (popc32(x[t] & z[t]) & 1) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t d = 0; d < S.dim; ++d) out[d] = 0.0;
    for (int64_t i = 0; i < n_in; ++i) {
        uint32_t b = sector_unrank(&S, in_idx[i]);
        for (int64_t t = 0; t < nterm; ++t) {
            uint32_t bo = b ^ x[t];
            if (!in_sector(&S, bo)) continue;
            int ny = popc32(x[t] & z[t]);
            double ph = ((ny / 2) & 1) ? -1.0 : 1.0;
            if (popc32(z[t] & b) & 1) ph = -ph;
            out[sector_rank(&S, bo)] += c[t] * ph * in_val[i];
        }
    }
    return 0;
}

double orc_dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------ excitations */

/*
 * Generator kind: 0 fermionic excitations (default), 1 qubit excitations
 * (the QEB pool of the paper's ADAPT-VQE description): the qubit operators
 * sigma^+ / sigma^- carry no Jordan-Wigner parity string, so every sign is +1.
 */
static int orc_qubit_exc = 0;
void orc_set_qubit_excitations(int on) { orc_qubit_exc = on ? 1 : 0; }

/*
 * tau = a+_{c1} a+_{c2} a_{a2} a_{a1}  (c1 < c2, a1 < a2)  or  a+_c a_a,
 * applied to the basis state b right to left; each ladder operator on qubit
 * q contributes (-1)^{popc(current & (2^q - 1))} (fermionic kind; +1 for
 * qubit excitations).  Returns 0 if tau b = 0, else the sign, and the
 * target in *out.
 */
int orc_apply_tau(uint32_t cre, uint32_t ann, uint32_t b, uint32_t *out) {
    int cq[2], aq[2], nc = 0, nan_ = 0;
    for (int q = 0; q < 32; ++q) {
        if (cre & (1u << q)) { if (nc < 2) cq[nc] = q; ++nc; }
        if (ann & (1u << q)) { if (nan_ < 2) aq[nan_] = q; ++nan_; }
    }
    if (nc != nan_ || nc < 1 || nc > 2) return 0;
    /* operator list in the order applied: a_{a1}, a_{a2}, a+_{c2}, a+_{c1} */
    int qs[4], cr[4], k = 0;
    qs[k] = aq[0]; cr[k++] = 0;
    if (nan_ == 2) { qs[k] = aq[1]; cr[k++] = 0; }
    if (nc == 2) { qs[k] = cq[1]; cr[k++] = 1; }
    qs[k] = cq[0]; cr[k++] = 1;
    int sign = 1;
    uint32_t cur = b;
    for (int i = 0; i < k; ++i) {
        uint32_t bit = 1u << qs[i];
        int occ = (cur & bit) != 0;
        if (cr[i] ? occ : !occ) return 0;
        if (!orc_qubit_exc && (popc32(cur & (bit - 1u)) & 1)) sign = -sign;
        cur ^= bit;
    }
    *out = cur;
    return sign;
}

/*
 * Pool gradients, one generator A_k = tau_k - tau_k^dagger at a time:
 * g_k = dE/dtheta at theta = 0 of <psi| e^{-theta A} H e^{theta A} |psi>
 *     = 2 <sigma| A_k psi>  with sigma = H psi,
 * summed literally over every sector state D with tau_k D != 0:
 * A|D> = s|D'>, A|D'> = -s|D>  =>  contribution 2 s (sigma[D'] psi[D] - sigma[D] psi[D']).
 * (ADAPT-VQE operator selection, paper "Numerical performance".)
 */
void orc_pool_gradients(int M, int na, int nb, int64_t nops, const uint32_t *cre,
                        const uint32_t *ann, const double *psi, const double *sigma,
                        double *grad) {
    sector_t S; sector_init(&S, M, na, nb);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nops; ++k) {
        double g = 0.0;
        for (int64_t d = 0; d < S.dim; ++d) {
            uint32_t b = sector_unrank(&S, d), bp;
            int s = orc_apply_tau(cre[k], ann[k], b, &bp);
            if (!s) continue;
            int64_t dp = sector_rank(&S, bp);
            g += 2.0 * s * (sigma[dp] * psi[d] - sigma[d] * psi[dp]);
        }
        grad[k] = g;
    }
}

/*
 * The same pool gradients when psi is given with the list of its nonzero
 * sector indices nz[0..n_nz) (psi and sigma still dense).  Every pair
 * (D, D' = tau D) of g_k = 2 sum s (sigma[D'] psi[D] - sigma[D] psi[D'])
 * whose D and D' both lie outside the list contributes exactly 0, so the sum
 * is split into its two halves and each is taken over the listed states only:
 *   2 sum_{b listed, tau b != 0}       s(b)  sigma[tau b]      psi[b]
 * - 2 sum_{b listed, tau^dag b != 0}   s'(b) sigma[tau^dag b] psi[b],
 * where tau^dag = a+_{a1} a+_{a2} a_{c2} a_{c1} is applied literally (the
 * excitation with creation and annihilation masks swapped) and its sign
 * s' = <tau^dag b| tau^dag |b> equals <b| tau |tau^dag b> (real matrix
 * elements).  A listed index must be a nonzero of psi, each listed once.
 */
void orc_pool_gradients_sparse(int M, int na, int nb, int64_t nops, const uint32_t *cre,
                               const uint32_t *ann, int64_t n_nz, const int64_t *nz,
                               const double *psi, const double *sigma, double *grad) {
    sector_t S; sector_init(&S, M, na, nb);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nops; ++k) {
        double g = 0.0;
        for (int64_t i = 0; i < n_nz; ++i) {
            int64_t d = nz[i];
            uint32_t b = sector_unrank(&S, d), bp;
            int s = orc_apply_tau(cre[k], ann[k], b, &bp);
            if (s) g += 2.0 * s * sigma[sector_rank(&S, bp)] * psi[d];
            s = orc_apply_tau(ann[k], cre[k], b, &bp);
            if (s) g -= 2.0 * s * sigma[sector_rank(&S, bp)] * psi[d];
        }
        grad[k] = g;
    }
}

/* out = A psi  (A = tau - tau^dagger), out must not alias psi */
void orc_apply_generator(int M, int na, int nb, uint32_t cre, uint32_t ann,
                         const double *psi, double *out) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int64_t d = 0; d < S.dim; ++d) out[d] = 0.0;
    for (int64_t d = 0; d < S.dim; ++d) {
        uint32_t b = sector_unrank(&S, d), bp;
        int s = orc_apply_tau(cre, ann, b, &bp);
        if (!s) continue;
        int64_t dp = sector_rank(&S, bp);
        out[dp] += s * psi[d];
        out[d] -= s * psi[dp];
    }
}

/*
 * psi <- exp(theta A) psi.  A^2 = -1 on each pair {D, D'} and 0 elsewhere,
 * so exp(theta A) = cos(theta) + sin(theta) A on the pair (the exponentiated
 * fermionic operator of "Sparse State-Vector Emulation").
 */
void orc_rotate(int M, int na, int nb, uint32_t cre, uint32_t ann, double theta, double *psi) {
    sector_t S; sector_init(&S, M, na, nb);
    double co = cos(theta), sn = sin(theta);
    for (int64_t d = 0; d < S.dim; ++d) {
        uint32_t b = sector_unrank(&S, d), bp;
        int s = orc_apply_tau(cre, ann, b, &bp);
        if (!s) continue;
        int64_t dp = sector_rank(&S, bp);
        double x0 = psi[d], x1 = psi[dp];
        psi[d] = co * x0 - s * sn * x1;
        psi[dp] = s * sn * x0 + co * x1;
    }
}

/* number of pairs |P_k| of a generator (states D with tau D != 0) */
int64_t orc_pair_count(int M, int na, int nb, uint32_t cre, uint32_t ann) {
    sector_t S; sector_init(&S, M, na, nb);
    int64_t n = 0;
    for (int64_t d = 0; d < S.dim; ++d) {
        uint32_t bp;
        if (orc_apply_tau(cre, ann, sector_unrank(&S, d), &bp)) ++n;
    }
    return n;
}

/* <n_q> = sum_D psi[D]^2 [q occupied in D] for all 2M spin-orbitals */
void orc_occupations(int M, int na, int nb, const double *psi, double *occ) {
    sector_t S; sector_init(&S, M, na, nb);
    for (int q = 0; q < 2 * M; ++q) occ[q] = 0.0;
    for (int64_t d = 0; d < S.dim; ++d) {
        uint32_t b = sector_unrank(&S, d);
        for (int q = 0; q < 2 * M; ++q)
            if (b & (1u << q)) occ[q] += psi[d] * psi[d];
    }
}

/* The pairs (D, D' = tau D, sign) of one generator, by literal application
 * of tau to every sector state; returns their number (arrays hold at least
 * orc_pair_count entries). */
int64_t orc_pair_list(int M, int na, int nb, uint32_t cre, uint32_t ann, int64_t *src, int64_t *dst,
                      int8_t *sign) {
    sector_t S; sector_init(&S, M, na, nb);
    int64_t n = 0;
    for (int64_t d = 0; d < S.dim; ++d) {
        uint32_t bp;
        int s = orc_apply_tau(cre, ann, sector_unrank(&S, d), &bp);
        if (!s) continue;
        src[n] = d;
        dst[n] = sector_rank(&S, bp);
        sign[n] = (int8_t)s;
        ++n;
    }
    return n;
}
