/*
 * FP64 CPU oracle for the ParaQAOA hot path (arXiv 2603.26232).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * HIP path is checked against. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library never links,
 * calls or includes anything from here, and this file includes nothing from
 * the product. It shares no code, tables or helpers with the GPU path.
 *
 * Conventions (paper Sec. 2.1, 2.2 and 3.3):
 *   - amplitude index z: bit j of z is local vertex j; bit value 1 puts the
 *     vertex in S (the bitstring picture of Sec. 2.4 / Fig. 2);
 *   - H_C = diag(C(z)), C(z) = sum over edges (u,v) of w_uv [z_u != z_v]:
 *     the Max-Cut objective of Sec. 2.1 as a diagonal Hamiltonian, which the
 *     QAOA of Sec. 2.2 maximises;
 *   - H_M = sum_j X_j (transverse field), U_C = e^{-i gamma H_C},
 *     U_M = e^{-i beta H_M} = prod_j (cos beta I - i sin beta X_j);
 *   - |psi(gamma,beta)> = U_M(b_p) U_C(g_p) ... U_M(b_1) U_C(g_1) |+>^n.
 * All floating point is IEEE double; no fast-math. Complex numbers are C99
 * `double complex` (two doubles, real then imaginary).
 *
 * Parity pins for every function are in the test-suite (closed forms,
 * symmetries, brute force, dense matrix exponentials); functions whose
 * results no pin fixes say "parity unpinned" below.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static inline int64_t weight_of(const int32_t* w, int64_t e) { return w ? (int64_t)w[e] : 1; }

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of threads the later parallel loops use (timing on one core). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: CutVal(x) = sum of w_uv over edges whose endpoints are on       */
/* different sides of the bipartition x (x[v] in {0,1}).                     */
/* ------------------------------------------------------------------------ */
int64_t or_cutval(int64_t nE, const int32_t* u, const int32_t* v, const int32_t* w,
                  const uint8_t* x)
{
    int64_t cut = 0;
    for (int64_t e = 0; e < nE; ++e)
        if (x[u[e]] != x[v[e]]) cut += weight_of(w, e);
    return cut;
}

/* CutVal for A assignments given bit-packed (vertex t = word t/32, bit t%32). */
void or_cutval_packed(int64_t A, int32_t nV, int64_t nE, const int32_t* u, const int32_t* v,
                      const int32_t* w, const uint32_t* words, int64_t* out)
{
    int64_t nw = (nV + 31) / 32;
    for (int64_t a = 0; a < A; ++a) {
        const uint32_t* x = words + a * nw;
        int64_t cut = 0;
        for (int64_t e = 0; e < nE; ++e) {
            int xu = (x[u[e] / 32] >> (u[e] % 32)) & 1;
            int xv = (x[v[e] / 32] >> (v[e] % 32)) & 1;
            if (xu != xv) cut += weight_of(w, e);
        }
        out[a] = cut;
    }
}

/* Exhaustive maximum cut (the optimum of Sec. 2.1, used as the AR
 * denominator for small graphs). Vertex 0 is fixed to side 0, which loses
 * nothing because CutVal(x) = CutVal(complement of x). */
int64_t or_bruteforce_maxcut(int32_t nV, int64_t nE, const int32_t* u, const int32_t* v,
                             const int32_t* w, uint8_t* best_x)
{
    uint8_t* x = (uint8_t*)calloc((size_t)nV, 1);
    int64_t best = -1;
    uint64_t count = (nV >= 1) ? (1ull << (nV - 1)) : 1;
    for (uint64_t m = 0; m < count; ++m) {
        x[0] = 0;
        for (int32_t t = 1; t < nV; ++t) x[t] = (uint8_t)((m >> (t - 1)) & 1);
        int64_t c = or_cutval(nE, u, v, w, x);
        if (c > best) {
            best = c;
            if (best_x) memcpy(best_x, x, (size_t)nV);
        }
    }
    free(x);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2: the diagonal of H_C for one subgraph of n vertices.             */
/* ------------------------------------------------------------------------ */
void or_cut_table(int32_t n, int64_t nE, const int32_t* u, const int32_t* v, const int32_t* w,
                  int64_t* C)
{
    uint64_t dim = 1ull << n;
    for (uint64_t z = 0; z < dim; ++z) {
        int64_t c = 0;
        for (int64_t e = 0; e < nE; ++e)
            if (((z >> u[e]) & 1) != ((z >> v[e]) & 1)) c += weight_of(w, e);
        C[z] = c;
    }
}

/* U_C(gamma)^sign: psi(z) <- e^{-i sign gamma C(z)} psi(z); the product
 * gamma * C(z) is formed in double. */
static void apply_cost(int32_t n, cplx* psi, const int64_t* C, double gamma, double sign)
{
    uint64_t dim = 1ull << n;
    for (uint64_t z = 0; z < dim; ++z) {
        double phi = sign * gamma * (double)C[z];
        psi[z] *= (cos(phi) - I * sin(phi));
    }
}

/* U_M(beta)^sign: for every qubit j the 2x2 rotation cos(beta) I -
 * i sign sin(beta) X on the amplitude pairs (z, z | 2^j), bit j of z zero. */
static void apply_mixer(int32_t n, cplx* psi, double beta, double sign)
{
    uint64_t dim = 1ull << n;
    double c = cos(beta), s = sign * sin(beta);
    for (int32_t j = 0; j < n; ++j) {
        uint64_t bit = 1ull << j;
        for (uint64_t z = 0; z < dim; ++z) {
            if (z & bit) continue;
            cplx a = psi[z], b = psi[z | bit];
            psi[z] = c * a - I * s * b;
            psi[z | bit] = -I * s * a + c * b;
        }
    }
}

/* |+>^n: every amplitude 2^{-n/2}. */
static void init_plus(int32_t n, cplx* psi)
{
    uint64_t dim = 1ull << n;
    double a = 1.0 / sqrt((double)dim);
    for (uint64_t z = 0; z < dim; ++z) psi[z] = a;
}

/* The QAOA ansatz state of Sec. 2.2 for angles gamma[0..p-1], beta[0..p-1]. */
void or_qaoa_state(int32_t n, const int64_t* C, int32_t p, const double* gamma,
                   const double* beta, cplx* psi)
{
    init_plus(n, psi);
    for (int32_t l = 0; l < p; ++l) {
        apply_cost(n, psi, C, gamma[l], +1.0);
        apply_mixer(n, psi, beta[l], +1.0);
    }
}

/* The inverse circuit, layer p down to 1 (used by a round-trip pin). */
void or_qaoa_unapply(int32_t n, const int64_t* C, int32_t p, const double* gamma,
                     const double* beta, cplx* psi)
{
    for (int32_t l = p - 1; l >= 0; --l) {
        apply_mixer(n, psi, beta[l], -1.0);
        apply_cost(n, psi, C, gamma[l], -1.0);
    }
}

/* Pairwise (cascade) sum of t[0..m-1]. */
static double pairwise_sum(const double* t, uint64_t m)
{
    if (m <= 8) {
        double s = 0.0;
        for (uint64_t i = 0; i < m; ++i) s += t[i];
        return s;
    }
    uint64_t h = m / 2;
    return pairwise_sum(t, h) + pairwise_sum(t + h, m - h);
}

/* The QAOA objective <psi|H_C|psi> = sum_z |psi(z)|^2 C(z) (Sec. 2.2). */
double or_expectation(int32_t n, const cplx* psi, const int64_t* C)
{
    uint64_t dim = 1ull << n;
    double* t = (double*)malloc(dim * sizeof(double));
    for (uint64_t z = 0; z < dim; ++z) {
        double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
        t[z] = pr * (double)C[z];
    }
    double e = pairwise_sum(t, dim);
    free(t);
    return e;
}

/* Free vertices of a subgraph: those without an edge of positive weight
 * inside it (bit j of the result for local vertex j). Flipping the bit of a
 * free vertex leaves C(z) unchanged, so its qubit stays in |+> through every
 * layer (|+> is an eigenvector of X, and U_C does not act on it): the state
 * is exactly invariant under that flip. */
uint32_t or_free_mask(int32_t n, int64_t ne, const int32_t* u, const int32_t* v, const int32_t* w)
{
    uint32_t busy = 0;
    for (int64_t e = 0; e < ne; ++e)
        if (weight_of(w, e) > 0) busy |= (1u << u[e]) | (1u << v[e]);
    uint32_t all = (n >= 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
    return all & ~busy;
}

/* Order of the strings inside a tie group: a bijection of [0, 2^m) built
 * from Marsaglia's xorshift step g(x) = x XOR (x >> s), s = ceil(m/2) (its
 * own inverse on m bits), and Knuth's multiplicative hashing by the odd
 * constant 2654435761 (2^32 / golden ratio): rank(x) = g(2654435761 g(x)
 * mod 2^m). Both steps are bijections, so ranks are distinct. */
static uint64_t xs_step(uint64_t x, int m)
{
    return x ^ (x >> ((m + 1) / 2));
}

static uint64_t hash_rank(uint64_t x, int m)
{
    if (m <= 0) return 0;
    uint64_t mask = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
    return xs_step((xs_step(x, m) * 2654435761ull) & mask, m);
}

/* rank of index x among the 2^m strings of a tie group (exported for tests) */
uint64_t or_tie_rank(uint64_t x, int32_t m)
{
    return hash_rank(x, m);
}

/* the bits of x at the positions of mask, packed to the low end */
static uint64_t gather_bits(uint64_t x, uint32_t mask)
{
    uint64_t out = 0;
    int k = 0;
    for (int j = 0; j < 32; ++j)
        if (mask & (1u << j)) {
            out |= ((x >> j) & 1ull) << k;
            ++k;
        }
    return out;
}

typedef struct {
    double pr;      /* probability of the tie group (that of its representative) */
    uint64_t rep;   /* the group's representative */
    uint64_t rank;  /* hash rank of the string inside its group */
    uint64_t z;
} topk_entry;

/* (pr desc, rep asc, rank asc) */
static int topk_before(const topk_entry* a, const topk_entry* b)
{
    if (a->pr != b->pr) return a->pr > b->pr;
    if (a->rep != b->rep) return a->rep < b->rep;
    return a->rank < b->rank;
}

/* Selective Distribution Exploration (Sec. 3.3.2): the K most probable
 * bitstrings, pi(z) = |psi(z)|^2 from the full distribution. With
 * `canonical` set only z whose bit 0 is 0 are candidates (pi(z) equals
 * pi(complement z) exactly, so this keeps one of each complement pair).
 *
 * Ties (the paper does not order equal probabilities). Besides the
 * complement, pi is exactly invariant under flipping the bit of any free
 * vertex (free_mask, see or_free_mask). The candidates that these moves
 * connect form a tie group of equal probability:
 *   Fm = the free vertices other than vertex 0 in canonical mode, all free
 *        vertices in raw mode;
 *   the partner move complements every bit and, in canonical mode, flips
 *        bit 0 back; it stays inside the candidates in raw mode, and in
 *        canonical mode when vertex 0 is free;
 *   r(z) = z with the bits of Fm cleared; if the partner move applies and
 *        the subgraph has a vertex that is not free, the group has two
 *        halves {r ^ S}, {r' ^ S} (S over Fm, r' = r of the partner) and its
 *        representative is min(r, r'); else one half and r itself.
 * A string's index inside its group is x = (bits of z at Fm, packed) with
 * the half as an extra low bit when there are two halves (m bits), and its
 * rank is hash_rank(x, m). Order: the group's probability (that of its
 * representative) descending, representative ascending, rank ascending.
 * Returns K_eff = min(k, #cand); the remaining rows of idx/prob are filled
 * with UINT32_MAX / -1. */
int32_t or_topk(int32_t n, const cplx* psi, int32_t k, int32_t canonical, uint32_t free_mask, uint32_t* idx,
                double* prob)
{
    uint64_t dim = 1ull << n;
    uint64_t all = dim - 1ull;
    uint32_t fm = canonical ? (free_mask & ~1u) : free_mask;
    int partner_ok = canonical ? (int)(free_mask & 1u) : 1;
    int halves = (partner_ok && (uint64_t)free_mask != all) ? 2 : 1;
    int m = __builtin_popcount(fm) + (halves == 2 ? 1 : 0);
    topk_entry* top = (topk_entry*)malloc((size_t)(k > 0 ? k : 1) * sizeof(topk_entry));
    int32_t have = 0;
    for (uint64_t z = 0; z < dim; ++z) {
        if (canonical && (z & 1)) continue;
        topk_entry e;
        uint64_t r = z & ~(uint64_t)fm;
        uint64_t half = 0;
        e.rep = r;
        if (halves == 2) {
            uint64_t pz = canonical ? ((~z & all) ^ 1ull) : (~z & all);
            uint64_t r2 = pz & ~(uint64_t)fm;
            if (r2 < r) {
                e.rep = r2;
                half = 1;
            }
        }
        uint64_t x = gather_bits(z, fm);
        if (halves == 2) x = (x << 1) | half;
        e.rank = hash_rank(x, m);
        e.pr = creal(psi[e.rep]) * creal(psi[e.rep]) + cimag(psi[e.rep]) * cimag(psi[e.rep]);
        e.z = z;
        /* insertion into the sorted top list */
        int32_t pos = have;
        while (pos > 0 && topk_before(&e, &top[pos - 1])) --pos;
        if (pos >= k) continue;
        int32_t last = (have < k) ? have : k - 1;
        for (int32_t q = last; q > pos; --q) top[q] = top[q - 1];
        top[pos] = e;
        if (have < k) ++have;
    }
    for (int32_t q = 0; q < k; ++q) {
        idx[q] = q < have ? (uint32_t)top[q].z : UINT32_MAX;
        prob[q] = q < have ? top[q].pr : -1.0;
    }
    free(top);
    return have;
}

/* Exact gradient of E(gamma, beta) = <psi|H_C|psi> by the adjoint sweep.
 * Forward to psi_p; lambda = C psi_p; then for l = p..1:
 *   dE/dbeta_l  = 2 Im <lambda| H_M |psi>   (both taken after U_M(beta_l))
 *   psi, lambda <- U_M(beta_l)^dagger applied to each
 *   dE/dgamma_l = 2 Im <lambda| H_C |psi>   (both taken after U_C(gamma_l))
 *   psi, lambda <- U_C(gamma_l)^dagger applied to each.
 * This follows from d/dtheta e^{-i theta H} = -i H e^{-i theta H} and
 * 2 Re(-i w) = 2 Im(w). */
void or_gradient(int32_t n, const int64_t* C, int32_t p, const double* gamma,
                 const double* beta, double* E, double* dgamma, double* dbeta)
{
    uint64_t dim = 1ull << n;
    cplx* psi = (cplx*)malloc(dim * sizeof(cplx));
    cplx* lam = (cplx*)malloc(dim * sizeof(cplx));
    or_qaoa_state(n, C, p, gamma, beta, psi);
    if (E) *E = or_expectation(n, psi, C);
    for (uint64_t z = 0; z < dim; ++z) lam[z] = (double)C[z] * psi[z];
    for (int32_t l = p - 1; l >= 0; --l) {
        /* <lambda|H_M|psi> = sum_j sum_z conj(lambda(z)) psi(z xor 2^j) */
        double acc = 0.0;
        for (int32_t j = 0; j < n; ++j) {
            uint64_t bit = 1ull << j;
            for (uint64_t z = 0; z < dim; ++z) acc += cimag(conj(lam[z]) * psi[z ^ bit]);
        }
        dbeta[l] = 2.0 * acc;
        apply_mixer(n, psi, beta[l], -1.0);
        apply_mixer(n, lam, beta[l], -1.0);
        acc = 0.0;
        for (uint64_t z = 0; z < dim; ++z) acc += cimag(conj(lam[z]) * (double)C[z] * psi[z]);
        dgamma[l] = 2.0 * acc;
        apply_cost(n, psi, C, gamma[l], -1.0);
        apply_cost(n, lam, C, gamma[l], -1.0);
    }
    free(psi);
    free(lam);
}

/* Cold-start angles: linear ramp gamma_l = (pi/2)(l - 1/2)/p,
 * beta_l = (pi/4)(1 - (l - 1/2)/p), l = 1..p (our reading; the paper only
 * says that initialisation matters, Sec. 2.2). */
void or_cold_start(int32_t p, double* gamma, double* beta)
{
    for (int32_t l = 0; l < p; ++l) {
        double f = ((double)l + 0.5) / (double)p;
        gamma[l] = 0.5 * M_PI * f;
        beta[l] = 0.25 * M_PI * (1.0 - f);
    }
}

/* Angle optimisation (Sec. 2.2 names gradient descent; our reading is Adam
 * on exact adjoint gradients, maximising E): for t = 1..T,
 *   g = grad E(theta); m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   theta += lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * E_hist[t] (t = 0..T-1) receives E at the start of step t, E_hist[T] the
 * final E, when E_hist is not NULL. Parity unpinned against the paper (it
 * gives no optimiser settings); pinned by a ring optimum and by gradient
 * checks. */
void or_adam_solve(int32_t n, const int64_t* C, int32_t p, int32_t T, double lr, double b1,
                   double b2, double eps, double* gamma, double* beta, double* E_hist)
{
    double m[64], v[64], g[64];
    for (int32_t i = 0; i < 2 * p; ++i) m[i] = v[i] = 0.0;
    for (int32_t t = 1; t <= T; ++t) {
        double E;
        or_gradient(n, C, p, gamma, beta, &E, g, g + p);
        if (E_hist) E_hist[t - 1] = E;
        double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
        for (int32_t i = 0; i < 2 * p; ++i) {
            m[i] = b1 * m[i] + (1.0 - b1) * g[i];
            v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
            double step = lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
            if (i < p) gamma[i] += step;
            else beta[i - p] += step;
        }
    }
    if (E_hist) {
        uint64_t dim = 1ull << n;
        cplx* psi = (cplx*)malloc(dim * sizeof(cplx));
        or_qaoa_state(n, C, p, gamma, beta, psi);
        E_hist[T] = or_expectation(n, psi, C);
        free(psi);
    }
}

/* One Adam step on a flat parameter vector (shared by the angle optimiser's
 * batch form and the MLP trainer), maximising when sign = +1 and minimising
 * when sign = -1. */
void or_adam_update(int64_t count, double* theta, const double* grad, double* m, double* v,
                    int32_t t, double lr, double b1, double b2, double eps, double sign)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < count; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        theta[i] += sign * lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Batched plain method for many subgraphs (OpenMP over subgraphs).          */
/* ------------------------------------------------------------------------ */

/* Evaluate the ansatz at fixed angles for a batch of subgraphs and return
 * E_b and the top-k lists. Subgraph b has nq[b] qubits and edges
 * eoff[b]..eoff[b+1]-1 of (u, v, w) in local ids. Angles row-major [b][l]. */
void or_eval_batch(int32_t B, const int32_t* nq, const int64_t* eoff, const int32_t* u,
                   const int32_t* v, const int32_t* w, int32_t p, const double* gamma,
                   const double* beta, double* E, int32_t k, int32_t canonical, uint32_t* idx,
                   double* prob)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; ++b) {
        int32_t n = nq[b];
        uint64_t dim = 1ull << n;
        int64_t e0 = eoff[b], ne = eoff[b + 1] - eoff[b];
        int64_t* C = (int64_t*)malloc(dim * sizeof(int64_t));
        cplx* psi = (cplx*)malloc(dim * sizeof(cplx));
        or_cut_table(n, ne, u + e0, v + e0, w ? w + e0 : NULL, C);
        or_qaoa_state(n, C, p, gamma + (int64_t)b * p, beta + (int64_t)b * p, psi);
        E[b] = or_expectation(n, psi, C);
        if (k > 0)
            or_topk(n, psi, k, canonical, or_free_mask(n, ne, u + e0, v + e0, w ? w + e0 : NULL),
                    idx + (int64_t)b * k, prob + (int64_t)b * k);
        free(C);
        free(psi);
    }
}

/* Full plain solve per subgraph: Adam for T steps from the given angles
 * (updated in place), then the final state's E and top-k. */
void or_solve_batch(int32_t B, const int32_t* nq, const int64_t* eoff, const int32_t* u,
                    const int32_t* v, const int32_t* w, int32_t p, int32_t T, double lr,
                    double b1, double b2, double eps, double* gamma, double* beta, double* E,
                    int32_t k, int32_t canonical, uint32_t* idx, double* prob)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; ++b) {
        int32_t n = nq[b];
        uint64_t dim = 1ull << n;
        int64_t e0 = eoff[b], ne = eoff[b + 1] - eoff[b];
        int64_t* C = (int64_t*)malloc(dim * sizeof(int64_t));
        cplx* psi = (cplx*)malloc(dim * sizeof(cplx));
        or_cut_table(n, ne, u + e0, v + e0, w ? w + e0 : NULL, C);
        double* g = gamma + (int64_t)b * p;
        double* be = beta + (int64_t)b * p;
        or_adam_solve(n, C, p, T, lr, b1, b2, eps, g, be, NULL);
        or_qaoa_state(n, C, p, g, be, psi);
        E[b] = or_expectation(n, psi, C);
        if (k > 0)
            or_topk(n, psi, k, canonical, or_free_mask(n, ne, u + e0, v + e0, w ? w + e0 : NULL),
                    idx + (int64_t)b * k, prob + (int64_t)b * k);
        free(C);
        free(psi);
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.2.2, Alg. 1 (Connectivity-Preserving Partitioning) under our       */
/* reading: subgraph i is the index range [start_i, start_i + size_i), the   */
/* next range starts at the last vertex of this one (exactly one shared      */
/* vertex), and the last range is clipped at |V|.                            */
/* ------------------------------------------------------------------------ */

/* Equal sizes N with stride N-1: M = ceil((|V|-1)/(N-1)). Returns M. */
int32_t or_partition_equal(int32_t nV, int32_t N, int32_t* start, int32_t* size)
{
    if (nV <= N) {
        start[0] = 0;
        size[0] = nV;
        return 1;
    }
    int32_t M = (nV - 1 + (N - 2)) / (N - 1);
    for (int32_t i = 0; i < M; ++i) {
        start[i] = i * (N - 1);
        int32_t end = start[i] + N;
        if (end > nV) end = nV;
        size[i] = end - start[i];
    }
    return M;
}

/* Chain with given sizes (drawn by the caller): consume sizes in order
 * until the chain reaches |V|. Returns M. */
int32_t or_partition_chain(int32_t nV, int32_t count, const int32_t* sizes, int32_t* start,
                           int32_t* size)
{
    int32_t s = 0, M = 0;
    for (int32_t i = 0; i < count; ++i) {
        int32_t n = sizes[i];
        start[M] = s;
        if (s + n >= nV) {
            size[M++] = nV - s;
            return M;
        }
        size[M++] = n;
        s += n - 1;
    }
    return -1; /* ran out of sizes */
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.4, Alg. 2: merge of the candidate sets B_i = {b_j, complement b_j} */
/* over the chain. A path picks one member of B_1, then one compatible       */
/* member of each later B_i: the member whose bit for the shared vertex      */
/* (local vertex 0) agrees with the path. Path order is the depth-first      */
/* order of Alg. 2: level 1 lists b_1, ~b_1, b_2, ~b_2, ...; later levels    */
/* list candidates by j. Its digits are (2j+o) at level 1 and j afterwards.  */
/*                                                                          */
/* W <= 0: exhaustive depth-first traversal, CutVal over all of E at each    */
/* leaf, strict '>' so the first maximum in traversal order wins (the leaf  */
/* test is applied after the last level is appended).                        */
/* W > 0: level-wise beam; after each level keep the W paths with the        */
/* largest partial cut (edges whose endpoints are both assigned), ties by    */
/* path order. Partial cuts grow by the edges completed at that level, the   */
/* cut decomposition of Sec. 3.4.1. Exact when W >= 2 K^(M-1).               */
/* Candidates: cand[i*K + j], j < K; UINT32_MAX marks padding (K_i = number  */
/* of leading non-padding entries). Returns the best cut; best_x[nV] and     */
/* best_digits[M] receive the winning path; *leaves the number of leaves     */
/* enumerated (exhaustive) or scored at the last level (beam).               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nV, M, K;
    const int32_t *start, *size;
    int64_t nE;
    const int32_t *u, *v, *w;
    const uint32_t* cand;
    int32_t* Ki;
} merge_ctx;

static void assign_level(const merge_ctx* c, int32_t i, uint32_t b, int32_t o, uint8_t* x)
{
    for (int32_t t = 0; t < c->size[i]; ++t)
        x[c->start[i] + t] = (uint8_t)(((b >> t) & 1u) ^ (uint32_t)o);
}

/* exhaustive DFS */
static void dfs(const merge_ctx* c, int32_t level, uint8_t* x, int32_t* digits, int64_t* best,
                uint8_t* best_x, int32_t* best_digits, double* leaves)
{
    if (level == c->M) {
        int64_t cut = or_cutval(c->nE, c->u, c->v, c->w, x);
        *leaves += 1.0;
        if (cut > *best) {
            *best = cut;
            memcpy(best_x, x, (size_t)c->nV);
            memcpy(best_digits, digits, (size_t)c->M * sizeof(int32_t));
        }
        return;
    }
    for (int32_t j = 0; j < c->Ki[level]; ++j) {
        uint32_t b = c->cand[(int64_t)level * c->K + j];
        if (level == 0) {
            for (int32_t o = 0; o < 2; ++o) {
                assign_level(c, 0, b, o, x);
                digits[0] = 2 * j + o;
                dfs(c, 1, x, digits, best, best_x, best_digits, leaves);
            }
        } else {
            int32_t o = (int32_t)((b & 1u) ^ x[c->start[level]]);
            assign_level(c, level, b, o, x);
            digits[level] = j;
            dfs(c, level + 1, x, digits, best, best_x, best_digits, leaves);
        }
    }
}

/* beam state: one path = partial cut + digits + assignment */
typedef struct {
    int64_t score;
    int32_t* digits;
    uint8_t* x;
} beam_path;

static int32_t g_sort_len;
static int cmp_paths(const void* pa, const void* pb)
{
    const beam_path* a = (const beam_path*)pa;
    const beam_path* b = (const beam_path*)pb;
    if (a->score != b->score) return a->score > b->score ? -1 : 1;
    for (int32_t i = 0; i < g_sort_len; ++i)
        if (a->digits[i] != b->digits[i]) return a->digits[i] < b->digits[i] ? -1 : 1;
    return 0;
}

/* cut of the edges completed at level i: max(u, v) is a vertex that first
 * appears in V_i (for i = 0 every vertex of V_0 is new). The edges of each
 * level are listed once up front (lvl_edges[lvl_off[i] .. lvl_off[i+1])). */
static int64_t completed_cut(const merge_ctx* c, const int64_t* lvl_off, const int64_t* lvl_edges, int32_t i,
                             const uint8_t* x)
{
    int64_t s = 0;
    for (int64_t q = lvl_off[i]; q < lvl_off[i + 1]; ++q) {
        int64_t e = lvl_edges[q];
        if (x[c->u[e]] != x[c->v[e]]) s += weight_of(c->w, e);
    }
    return s;
}

static int32_t first_level(const merge_ctx* c, int32_t vtx)
{
    for (int32_t i = 0; i < c->M; ++i) {
        int32_t lo = (i == 0) ? c->start[0] : c->start[i] + 1;
        if (vtx >= lo && vtx < c->start[i] + c->size[i]) return i;
    }
    return -1;
}

int64_t or_merge(int32_t nV, int32_t M, const int32_t* start, const int32_t* size, int64_t nE,
                 const int32_t* u, const int32_t* v, const int32_t* w, int32_t K,
                 const uint32_t* cand, int64_t W, uint8_t* best_x, int32_t* best_digits,
                 double* leaves)
{
    merge_ctx c = {nV, M, K, start, size, nE, u, v, w, cand, NULL};
    /* chain sanity: contiguous ranges sharing exactly one vertex, covering V */
    if (M < 1 || start[0] != 0 || start[M - 1] + size[M - 1] != nV) return -1;
    for (int32_t i = 1; i < M; ++i)
        if (start[i] != start[i - 1] + size[i - 1] - 1) return -1;
    c.Ki = (int32_t*)malloc((size_t)M * sizeof(int32_t));
    for (int32_t i = 0; i < M; ++i) {
        int32_t k = 0;
        while (k < K && cand[(int64_t)i * K + k] != UINT32_MAX) ++k;
        c.Ki[i] = k;
        if (k == 0) {
            free(c.Ki);
            return -1;
        }
    }
    *leaves = 0.0;
    int64_t best = -1;
    if (W <= 0) {
        uint8_t* x = (uint8_t*)calloc((size_t)nV, 1);
        int32_t* digits = (int32_t*)calloc((size_t)M, sizeof(int32_t));
        dfs(&c, 0, x, digits, &best, best_x, best_digits, leaves);
        free(x);
        free(digits);
        free(c.Ki);
        return best;
    }
    /* beam: bucket the edges by the level that completes them */
    int64_t* lvl_off = (int64_t*)calloc((size_t)M + 1, sizeof(int64_t));
    int64_t* lvl_edges = (int64_t*)malloc((size_t)(nE > 0 ? nE : 1) * sizeof(int64_t));
    int32_t* lvl_of = (int32_t*)malloc((size_t)(nE > 0 ? nE : 1) * sizeof(int32_t));
    for (int64_t e = 0; e < nE; ++e) {
        int32_t mx = u[e] > v[e] ? u[e] : v[e];
        lvl_of[e] = first_level(&c, mx);
        lvl_off[lvl_of[e] + 1] += 1;
    }
    for (int32_t i = 0; i < M; ++i) lvl_off[i + 1] += lvl_off[i];
    {
        int64_t* fill = (int64_t*)malloc(((size_t)M + 1) * sizeof(int64_t));
        memcpy(fill, lvl_off, ((size_t)M + 1) * sizeof(int64_t));
        for (int64_t e = 0; e < nE; ++e) lvl_edges[fill[lvl_of[e]]++] = e;
        free(fill);
    }
    /* level 1 creates 2 K paths, later levels at most W K */
    int64_t cap = W * (int64_t)K;
    if (cap < 2 * (int64_t)K) cap = 2 * (int64_t)K;
    beam_path* cur = (beam_path*)calloc((size_t)cap, sizeof(beam_path));
    beam_path* nxt = (beam_path*)calloc((size_t)cap, sizeof(beam_path));
    for (int64_t r = 0; r < cap; ++r) {
        cur[r].digits = (int32_t*)calloc((size_t)M, sizeof(int32_t));
        cur[r].x = (uint8_t*)calloc((size_t)nV, 1);
        nxt[r].digits = (int32_t*)calloc((size_t)M, sizeof(int32_t));
        nxt[r].x = (uint8_t*)calloc((size_t)nV, 1);
    }
    int64_t ncur = 0;
    for (int32_t j = 0; j < c.Ki[0]; ++j)
        for (int32_t o = 0; o < 2; ++o) {
            beam_path* q = &nxt[ncur++];
            assign_level(&c, 0, cand[j], o, q->x);
            q->digits[0] = 2 * j + o;
            q->score = completed_cut(&c, lvl_off, lvl_edges, 0, q->x);
        }
    for (int32_t i = 0;; ++i) {
        g_sort_len = i + 1;
        qsort(nxt, (size_t)ncur, sizeof(beam_path), cmp_paths);
        if (ncur > W) ncur = W;
        beam_path* t = cur;
        cur = nxt;
        nxt = t;
        if (i == M - 1) break;
        int64_t nn = 0;
        int32_t lvl = i + 1;
        for (int64_t r = 0; r < ncur; ++r)
            for (int32_t j = 0; j < c.Ki[lvl]; ++j) {
                beam_path* q = &nxt[nn++];
                uint32_t b = cand[(int64_t)lvl * K + j];
                memcpy(q->x, cur[r].x, (size_t)nV);
                memcpy(q->digits, cur[r].digits, (size_t)M * sizeof(int32_t));
                int32_t o = (int32_t)((b & 1u) ^ q->x[start[lvl]]);
                assign_level(&c, lvl, b, o, q->x);
                q->digits[lvl] = j;
                q->score = cur[r].score + completed_cut(&c, lvl_off, lvl_edges, lvl, q->x);
            }
        ncur = nn;
        if (lvl == M - 1) *leaves = (double)nn;
    }
    if (M == 1) *leaves = (double)(2 * c.Ki[0]);
    best = cur[0].score;
    memcpy(best_x, cur[0].x, (size_t)nV);
    memcpy(best_digits, cur[0].digits, (size_t)M * sizeof(int32_t));
    for (int64_t r = 0; r < cap; ++r) {
        free(cur[r].digits);
        free(cur[r].x);
        free(nxt[r].digits);
        free(nxt[r].x);
    }
    free(cur);
    free(nxt);
    free(c.Ki);
    free(lvl_off);
    free(lvl_edges);
    free(lvl_of);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Angle predictor (not in the paper; a learned warm start for the angle     */
/* optimisation whose initialisation Sec. 2.2 says matters): a multilayer    */
/* perceptron in -> H -> H -> out with ReLU hidden layers and a linear       */
/* output. Parameters, flat, row-major: W1[H][in], b1[H], W2[H][H], b2[H],   */
/* W3[out][H], b3[out]. Loss = mean over batch and outputs of (y - t)^2.     */
/* FP64 throughout. Pinned by central finite differences.                    */
/* ------------------------------------------------------------------------ */
int64_t or_mlp_num_params(int32_t in, int32_t H, int32_t out)
{
    return (int64_t)H * in + H + (int64_t)H * H + H + (int64_t)out * H + out;
}

static void mlp_one(int32_t in, int32_t H, int32_t out, const double* P, const double* x, double* h1, double* h2,
                    double* y)
{
    const double* W1 = P;
    const double* b1 = W1 + (int64_t)H * in;
    const double* W2 = b1 + H;
    const double* b2 = W2 + (int64_t)H * H;
    const double* W3 = b2 + H;
    const double* b3 = W3 + (int64_t)out * H;
    for (int32_t i = 0; i < H; ++i) {
        double a = b1[i];
        for (int32_t f = 0; f < in; ++f) a += W1[(int64_t)i * in + f] * x[f];
        h1[i] = a > 0.0 ? a : 0.0;
    }
    for (int32_t i = 0; i < H; ++i) {
        double a = b2[i];
        for (int32_t j = 0; j < H; ++j) a += W2[(int64_t)i * H + j] * h1[j];
        h2[i] = a > 0.0 ? a : 0.0;
    }
    for (int32_t o = 0; o < out; ++o) {
        double a = b3[o];
        for (int32_t j = 0; j < H; ++j) a += W3[(int64_t)o * H + j] * h2[j];
        y[o] = a;
    }
}

void or_mlp_forward(int32_t B, int32_t in, int32_t H, int32_t out, const double* P, const double* X, double* Y)
{
    double* h1 = (double*)malloc((size_t)H * sizeof(double));
    double* h2 = (double*)malloc((size_t)H * sizeof(double));
    for (int32_t s = 0; s < B; ++s) mlp_one(in, H, out, P, X + (int64_t)s * in, h1, h2, Y + (int64_t)s * out);
    free(h1);
    free(h2);
}

/* loss and its gradient with respect to every parameter (back-propagation) */
double or_mlp_loss_grad(int32_t B, int32_t in, int32_t H, int32_t out, const double* P, const double* X,
                        const double* T, double* G)
{
    int64_t np = or_mlp_num_params(in, H, out);
    for (int64_t i = 0; i < np; ++i) G[i] = 0.0;
    const double* W2 = P + (int64_t)H * in + H;
    const double* W3 = W2 + (int64_t)H * H + H;
    double* gW1 = G;
    double* gb1 = gW1 + (int64_t)H * in;
    double* gW2 = gb1 + H;
    double* gb2 = gW2 + (int64_t)H * H;
    double* gW3 = gb2 + H;
    double* gb3 = gW3 + (int64_t)out * H;
    double* h1 = (double*)malloc((size_t)H * sizeof(double));
    double* h2 = (double*)malloc((size_t)H * sizeof(double));
    double* y = (double*)malloc((size_t)out * sizeof(double));
    double* d3 = (double*)malloc((size_t)out * sizeof(double));
    double* d2 = (double*)malloc((size_t)H * sizeof(double));
    double* d1 = (double*)malloc((size_t)H * sizeof(double));
    double loss = 0.0;
    const double scale = 1.0 / ((double)B * (double)out);
    for (int32_t s = 0; s < B; ++s) {
        const double* x = X + (int64_t)s * in;
        const double* t = T + (int64_t)s * out;
        mlp_one(in, H, out, P, x, h1, h2, y);
        for (int32_t o = 0; o < out; ++o) {
            double r = y[o] - t[o];
            loss += r * r * scale;
            d3[o] = 2.0 * r * scale;
        }
        for (int32_t j = 0; j < H; ++j) {
            double a = 0.0;
            for (int32_t o = 0; o < out; ++o) a += W3[(int64_t)o * H + j] * d3[o];
            d2[j] = h2[j] > 0.0 ? a : 0.0;
        }
        for (int32_t j = 0; j < H; ++j) {
            double a = 0.0;
            for (int32_t i = 0; i < H; ++i) a += W2[(int64_t)i * H + j] * d2[i];
            d1[j] = h1[j] > 0.0 ? a : 0.0;
        }
        for (int32_t o = 0; o < out; ++o) {
            for (int32_t j = 0; j < H; ++j) gW3[(int64_t)o * H + j] += d3[o] * h2[j];
            gb3[o] += d3[o];
        }
        for (int32_t i = 0; i < H; ++i) {
            for (int32_t j = 0; j < H; ++j) gW2[(int64_t)i * H + j] += d2[i] * h1[j];
            gb2[i] += d2[i];
        }
        for (int32_t i = 0; i < H; ++i) {
            for (int32_t f = 0; f < in; ++f) gW1[(int64_t)i * in + f] += d1[i] * x[f];
            gb1[i] += d1[i];
        }
    }
    free(h1);
    free(h2);
    free(y);
    free(d3);
    free(d2);
    free(d1);
    return loss;
}
