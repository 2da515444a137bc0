/*
 * CPU oracle for C := C + A.B mod p on Morton-hybrid operands.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the bench's CPU
 * baseline leg load it.  It shares no source, header, table or helper with
 * the HIP path.
 *
 * Every routine is written for obviousness, not speed: loops in the order the
 * definitions state, 128-bit accumulators, one reduction mod p at the end.
 *
 * Notation.  The paper writes the product as S_A = S_B . S_C with A as the
 * output (section 2, problem statement) and the accumulating form
 * S'_A += S'_B . S'_C (section 2.2).  Here, as in the library, the output is
 * C and the factors are A (m x k, left) and B (k x n, right).
 *
 * Contents
 *   oracle_matmul_modp          the definition of the product (Cartesian)
 *   oracle_matmul_modp_sub      the subtractive update C - A.B mod p
 *   oracle_matmul_modp_entries  the same definition, for chosen entries only
 *   oracle_freivalds            Freivalds' randomised product check
 *   oracle_mh_encode/_extract   Morton-hybrid index by walking the quadrant
 *                               recursion (section 2.2 Step 1 offsets,
 *                               Prop. 2.5 row-major offset inside a tile)
 *   oracle_mh_from/to_cartesian layout conversion through the encoder
 *   oracle_classify             brute-force aligned / contained / quadrant
 *   oracle_recursive_mm         the paper's modified sub-matrix product,
 *                               Steps 1-4 of section 2.2, on MH buffers
 *   oracle_limb_digits          balanced base-256 digits of a centred residue
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC mh_oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* The product, by definition.                                              */
/* ------------------------------------------------------------------------ */

/*
 * C[i][j] <- (C[i][j] + sum_{l<k} A[i][l] * B[l][j]) mod p for i<m, j<n.
 * Section 2 states the problem (a product of sub-matrices of Morton-hybrid
 * parents); section 2.2 writes it in accumulating form (+=).  Arrays are
 * Cartesian row-major uint32 with leading dimensions ldc, lda, ldb; entries
 * are residues in [0,p).  Each product is < 2^62 and k < 2^40, so the 128-bit
 * row accumulator cannot wrap.  i-l-j loop order; rows split over threads.
 */
void oracle_matmul_modp(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                        const uint32_t *B, int64_t ldb, int64_t m, int64_t k,
                        int64_t n, uint32_t p, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        u128 *acc = (u128 *)malloc(sizeof(u128) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) acc[j] = 0;
            for (int64_t l = 0; l < k; ++l) {
                uint64_t a = A[i * lda + l];
                const uint32_t *brow = B + l * ldb;
                for (int64_t j = 0; j < n; ++j) acc[j] += (u128)(a * (uint64_t)brow[j]);
            }
            for (int64_t j = 0; j < n; ++j) {
                u128 s = acc[j] + (u128)C[i * ldc + j];
                C[i * ldc + j] = (uint32_t)(s % p);
            }
        }
        free(acc);
    }
}

/*
 * The subtractive update C[i][j] <- (C[i][j] - sum_l A[i][l] B[l][j]) mod p,
 * the Schur complement step of an elimination.  The sum is reduced mod p
 * first, then subtracted as (C + p - s) mod p.
 */
void oracle_matmul_modp_sub(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                            const uint32_t *B, int64_t ldb, int64_t m, int64_t k, int64_t n,
                            uint32_t p, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        u128 *acc = (u128 *)malloc(sizeof(u128) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) acc[j] = 0;
            for (int64_t l = 0; l < k; ++l) {
                uint64_t a = A[i * lda + l];
                const uint32_t *brow = B + l * ldb;
                for (int64_t j = 0; j < n; ++j) acc[j] += (u128)(a * (uint64_t)brow[j]);
            }
            for (int64_t j = 0; j < n; ++j) {
                uint64_t s = (uint64_t)(acc[j] % p);
                C[i * ldc + j] = (uint32_t)(((uint64_t)C[i * ldc + j] + p - s) % p);
            }
        }
        free(acc);
    }
}

/*
 * The same definition evaluated for a list of entries (ri[q], cj[q]) only:
 * out[q] = (C[ri][cj] + sum_l A[ri][l] B[l][cj]) mod p.  C is read, not
 * written.  Used to check outputs of products too large for the full loop.
 */
void oracle_matmul_modp_entries(uint32_t *out, const int64_t *ri, const int64_t *cj,
                                int64_t count, const uint32_t *C, int64_t ldc,
                                const uint32_t *A, int64_t lda, const uint32_t *B,
                                int64_t ldb, int64_t k, uint32_t p, int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4)
    for (int64_t q = 0; q < count; ++q) {
        u128 s = C[ri[q] * ldc + cj[q]];
        for (int64_t l = 0; l < k; ++l)
            s += (u128)((uint64_t)A[ri[q] * lda + l] * (uint64_t)B[l * ldb + cj[q]]);
        out[q] = (uint32_t)(s % p);
    }
}

/*
 * Freivalds' check that Cnew = Cold + A.B (mod p): with x a vector of n
 * residues supplied by the caller, compare Cnew.x with Cold.x + A.(B.x), all
 * mod p.  Returns 1 if they agree.  A wrong Cnew passes with probability at
 * most 1/p per independent x.
 */
int oracle_freivalds(const uint32_t *Cnew, const uint32_t *Cold, int64_t ldc,
                     const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
                     int64_t m, int64_t k, int64_t n, uint32_t p, const uint32_t *x,
                     int nthreads)
{
    if (nthreads <= 0) nthreads = 1;
    uint64_t *bx = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k > 0 ? k : 1));
    int ok = 1;
#pragma omp parallel for num_threads(nthreads)
    for (int64_t l = 0; l < k; ++l) {
        u128 s = 0;
        for (int64_t j = 0; j < n; ++j) s += (u128)((uint64_t)B[l * ldb + j] * x[j]);
        bx[l] = (uint64_t)(s % p);
    }
#pragma omp parallel for num_threads(nthreads) reduction(&& : ok)
    for (int64_t i = 0; i < m; ++i) {
        u128 lhs = 0, rhs = 0;
        for (int64_t j = 0; j < n; ++j) {
            lhs += (u128)((uint64_t)Cnew[i * ldc + j] * x[j]);
            rhs += (u128)((uint64_t)Cold[i * ldc + j] * x[j]);
        }
        for (int64_t l = 0; l < k; ++l) rhs += (u128)((uint64_t)A[i * lda + l] * bx[l]);
        ok = ok && ((lhs % p) == (rhs % p));
    }
    free(bx);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Morton-hybrid index, by walking the recursion.                           */
/* ------------------------------------------------------------------------ */

/*
 * Index of Cartesian (i,j) in an N x N Morton-hybrid matrix with tile edge T
 * (N = T * 2^q).  Section 1: the Z (Morton) order recursion stops at T x T
 * sub-matrices, which are stored row-major.  Section 2.2 Step 1: the
 * quadrants of a block with first index alpha and lambda elements are laid
 * out NW, NE, SW, SE, starting at alpha, alpha + lambda/4, alpha + lambda/2,
 * alpha + 3 lambda/4.  Prop. 2.5: inside a tile with first index sigma the
 * entry at row offset i and column offset j sits at sigma + i T + j.
 */
uint64_t oracle_mh_encode(uint64_t i, uint64_t j, uint64_t T, uint64_t N)
{
    uint64_t alpha = 0, lambda = N * N, size = N;
    while (size > T) {
        uint64_t half = size / 2, quarter = lambda / 4, t = 0;
        if (i >= half) { t += 2; i -= half; }   /* south */
        if (j >= half) { t += 1; j -= half; }   /* east  */
        alpha += t * quarter;                   /* NW=0, NE=1, SW=2, SE=3 */
        lambda = quarter;
        size = half;
    }
    return alpha + i * T + j;
}

/* Inverse of oracle_mh_encode (the paper's extract_i, extract_j). */
void oracle_mh_extract(uint64_t z, uint64_t T, uint64_t N, uint64_t *i_out, uint64_t *j_out)
{
    uint64_t alpha = 0, lambda = N * N, size = N, i = 0, j = 0;
    while (size > T) {
        uint64_t half = size / 2, quarter = lambda / 4;
        uint64_t t = (z - alpha) / quarter;
        if (t & 2) i += half;
        if (t & 1) j += half;
        alpha += t * quarter;
        lambda = quarter;
        size = half;
    }
    i += (z - alpha) / T;
    j += (z - alpha) % T;
    *i_out = i;
    *j_out = j;
}

/* dst (N*N words, Morton-hybrid) <- src (Cartesian, row length ld). */
void oracle_mh_from_cartesian(uint32_t *dst, const uint32_t *src, int64_t ld,
                              int64_t N, int64_t T)
{
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            dst[oracle_mh_encode((uint64_t)i, (uint64_t)j, (uint64_t)T, (uint64_t)N)] =
                src[i * ld + j];
}

/* dst (Cartesian, row length ld) <- src (N*N words, Morton-hybrid). */
void oracle_mh_to_cartesian(uint32_t *dst, int64_t ld, const uint32_t *src,
                            int64_t N, int64_t T)
{
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            dst[i * ld + j] =
                src[oracle_mh_encode((uint64_t)i, (uint64_t)j, (uint64_t)T, (uint64_t)N)];
}

/* ------------------------------------------------------------------------ */
/* Classification by brute force.                                           */
/* ------------------------------------------------------------------------ */

#define ORACLE_ALIGNED 1u
#define ORACLE_CONTAINED 2u
#define ORACLE_QUADRANT 4u

static int is_pow2_multiple(int64_t x, int64_t T)
{
    if (x <= 0 || x % T) return 0;
    int64_t q = x / T;
    return (q & (q - 1)) == 0;
}

/* Is (row, col, size x size) one of the blocks met by the quadrant recursion
 * of the block at (r0, c0) with edge `edge`?  Enumerates the recursion. */
static int is_recursion_node(int64_t r0, int64_t c0, int64_t edge, int64_t T,
                             int64_t row, int64_t col, int64_t rows, int64_t cols)
{
    if (r0 == row && c0 == col && edge == rows && edge == cols) return 1;
    if (edge <= T) return 0;
    int64_t h = edge / 2;
    for (int t = 0; t < 4; ++t)
        if (is_recursion_node(r0 + (t >> 1) * h, c0 + (t & 1) * h, h, T, row, col, rows, cols))
            return 1;
    return 0;
}

/*
 * Flags of the block with first entry (row, col) and size rows x cols in an
 * N x N Morton-hybrid parent with tile edge T.
 *  ALIGNED   (Def. "aligned", section 2): it begins at the first entry of a
 *            row-major T x T sub-matrix and is 2^a T x 2^b T.  The first
 *            entry of a tile is the one whose index is a multiple of T^2.
 *  CONTAINED (Def. "contained", section 2.1): all of its entries lie in one
 *            row-major T x T sub-matrix, i.e. share one index / T^2.
 *  QUADRANT  it is the whole parent or one of the blocks produced by the
 *            repeated quadrant division of section 2.2 Step 1 (so that its
 *            entries form one index range [alpha, alpha + lambda)).
 * Every entry of the block is visited through the encoder.
 */
uint32_t oracle_classify(int64_t N, int64_t T, int64_t row, int64_t col,
                         int64_t rows, int64_t cols)
{
    uint32_t f = 0;
    if (rows <= 0 || cols <= 0) return 0;
    uint64_t first = oracle_mh_encode((uint64_t)row, (uint64_t)col, (uint64_t)T, (uint64_t)N);
    if (first % (uint64_t)(T * T) == 0 && is_pow2_multiple(rows, T) && is_pow2_multiple(cols, T))
        f |= ORACLE_ALIGNED;
    int contained = 1;
    uint64_t tile0 = first / (uint64_t)(T * T);
    for (int64_t i = row; i < row + rows && contained; ++i)
        for (int64_t j = col; j < col + cols; ++j)
            if (oracle_mh_encode((uint64_t)i, (uint64_t)j, (uint64_t)T, (uint64_t)N) /
                    (uint64_t)(T * T) != tile0) {
                contained = 0;
                break;
            }
    if (contained) f |= ORACLE_CONTAINED;
    if (is_recursion_node(0, 0, N, T, row, col, rows, cols)) f |= ORACLE_QUADRANT;
    return f;
}

/* ------------------------------------------------------------------------ */
/* The paper's modified sub-matrix product, Steps 1-4 of section 2.2.       */
/* ------------------------------------------------------------------------ */

/*
 * An aligned block M^k is (alpha, lambda): its first index and size
 * (section 2.2, the 3-tuple).  A sub-matrix S_{M^k} is (sigma, r, c): first
 * index and dimensions (the 4-tuple).  To carry out Step 4 each piece also
 * records where it sits in the product: (pr, pc) is the product coordinate
 * of its first entry, in the two product dimensions the operand spans
 * (C: i,j; A: i,l; B: l,j).  The paper notes the first entry of each S'
 * sits at row/column offset 0 or r_N / c_W from that of S (Step 2); pr, pc
 * follow the same offsets.
 */
typedef struct { uint64_t alpha, lambda; } blk_t;
typedef struct { uint64_t sigma; int64_t r, c, pr, pc; } sub_t;

typedef struct {
    uint32_t *C; const uint32_t *A, *B;
    uint64_t NC, NA, NB, T;
    uint32_t p;
    int count_only;
    uint64_t leaves;
} rec_ctx;

/*
 * Steps 1 and 2 for one operand: the (up to) four quadrants of the aligned
 * block and the part S' of S inside each.  A block that is already one
 * T x T tile is not divided (Prop. 2.3: a dimension stops at T); it is
 * returned as its own single "quadrant".  Returns the number of quadrants.
 */
static int split_operand(blk_t M, sub_t S, uint64_t T, uint64_t N, blk_t q[4], sub_t s[4])
{
    if (M.lambda == T * T) {
        q[0] = M;
        s[0] = S;
        return 1;
    }
    /* Step 1 */
    uint64_t lq = M.lambda / 4;
    for (int t = 0; t < 4; ++t) { q[t].alpha = M.alpha + (uint64_t)t * lq; q[t].lambda = lq; }
    /* Step 2 */
    uint64_t e_ne = M.alpha + 2 * lq - 1, e_sw = M.alpha + 3 * lq - 1;
    uint64_t i_s, j_s, i_ne, j_ne, i_sw, j_sw;
    oracle_mh_extract(S.sigma, T, N, &i_s, &j_s);
    oracle_mh_extract(e_ne, T, N, &i_ne, &j_ne);
    oracle_mh_extract(e_sw, T, N, &i_sw, &j_sw);
    int64_t rN = (int64_t)i_ne - (int64_t)i_s + 1;
    int64_t cW = (int64_t)j_sw - (int64_t)j_s + 1;
    /* r_N <= 0 (or c_W <= 0) means no part in the north (west) half; the
     * counts are also capped by the sub-matrix size. */
    if (rN < 0) rN = 0;
    if (rN > S.r) rN = S.r;
    if (cW < 0) cW = 0;
    if (cW > S.c) cW = S.c;
    int64_t rS = S.r - rN, cE = S.c - cW;
    int64_t rr[4] = {rN, rN, rS, rS}, cc[4] = {cW, cE, cW, cE};
    int64_t fr[4] = {0, 0, rN, rN}, fc[4] = {0, cW, 0, cW};
    for (int t = 0; t < 4; ++t) {
        s[t].r = rr[t];
        s[t].c = cc[t];
        s[t].pr = S.pr + fr[t];
        s[t].pc = S.pc + fc[t];
        s[t].sigma = (rr[t] > 0 && cc[t] > 0)
                         ? oracle_mh_encode(i_s + (uint64_t)fr[t], j_s + (uint64_t)fc[t], T, N)
                         : 0;
    }
    return 4;
}

/* The part of S covering product rows [r0, r0+nr) and columns [c0, c0+nc). */
static sub_t extract_part(sub_t S, int64_t r0, int64_t nr, int64_t c0, int64_t nc,
                          uint64_t T, uint64_t N)
{
    uint64_t i_s, j_s;
    oracle_mh_extract(S.sigma, T, N, &i_s, &j_s);
    sub_t out;
    out.r = nr;
    out.c = nc;
    out.pr = r0;
    out.pc = c0;
    out.sigma = oracle_mh_encode(i_s + (uint64_t)(r0 - S.pr), j_s + (uint64_t)(c0 - S.pc), T, N);
    return out;
}

static void intersect(int64_t a0, int64_t an, int64_t b0, int64_t bn, int64_t *o0, int64_t *on)
{
    int64_t lo = a0 > b0 ? a0 : b0;
    int64_t hi = (a0 + an) < (b0 + bn) ? (a0 + an) : (b0 + bn);
    *o0 = lo;
    *on = hi > lo ? hi - lo : 0;
}

/* Base case: all three pieces are contained in one row-major tile each, so
 * every entry is addressed as sigma + i T + j (Prop. 2.5). */
static void base_case(rec_ctx *x, sub_t SC, sub_t SA, sub_t SB)
{
    x->leaves++;
    if (x->count_only) return;
    uint64_t T = x->T;
    for (int64_t i = 0; i < SC.r; ++i)
        for (int64_t j = 0; j < SC.c; ++j) {
            u128 s = x->C[SC.sigma + (uint64_t)i * T + (uint64_t)j];
            for (int64_t l = 0; l < SA.c; ++l)
                s += (u128)((uint64_t)x->A[SA.sigma + (uint64_t)i * T + (uint64_t)l] *
                            (uint64_t)x->B[SB.sigma + (uint64_t)l * T + (uint64_t)j]);
            x->C[SC.sigma + (uint64_t)i * T + (uint64_t)j] = (uint32_t)(s % x->p);
        }
}

static void rec_mm(rec_ctx *x, blk_t Ck, sub_t SC, blk_t Ak, sub_t SA, blk_t Bk, sub_t SB)
{
    if (SC.r <= 0 || SC.c <= 0 || SA.c <= 0) return;
    uint64_t T = x->T;
    if (Ck.lambda == T * T && Ak.lambda == T * T && Bk.lambda == T * T) {
        base_case(x, SC, SA, SB);
        return;
    }
    blk_t qc[4], qa[4], qb[4];
    sub_t sc[4], sa[4], sb[4];
    int nc = split_operand(Ck, SC, T, x->NC, qc, sc);
    int na = split_operand(Ak, SA, T, x->NA, qa, sa);
    int nb = split_operand(Bk, SB, T, x->NB, qb, sb);
    /* Step 3: every combination (t,u,v) of quadrants (up to 64). */
    for (int t = 0; t < nc; ++t) {
        if (sc[t].r <= 0 || sc[t].c <= 0) continue;
        for (int u = 0; u < na; ++u) {
            if (sa[u].r <= 0 || sa[u].c <= 0) continue;
            for (int v = 0; v < nb; ++v) {
                if (sb[v].r <= 0 || sb[v].c <= 0) continue;
                /* Step 4: the compatible parts.  S'_C covers product rows
                 * I_C and columns J_C, S'_A rows I_A and inner range L_A,
                 * S'_B inner range L_B and columns J_B.  Their product is a
                 * part of the whole one on I_C n I_A, L_A n L_B, J_C n J_B. */
                int64_t i0, ni, l0, nl, j0, nj;
                intersect(sc[t].pr, sc[t].r, sa[u].pr, sa[u].r, &i0, &ni);
                intersect(sa[u].pc, sa[u].c, sb[v].pr, sb[v].r, &l0, &nl);
                intersect(sc[t].pc, sc[t].c, sb[v].pc, sb[v].c, &j0, &nj);
                if (ni <= 0 || nl <= 0 || nj <= 0) continue;
                sub_t pc = extract_part(sc[t], i0, ni, j0, nj, T, x->NC);
                sub_t pa = extract_part(sa[u], i0, ni, l0, nl, T, x->NA);
                sub_t pb = extract_part(sb[v], l0, nl, j0, nj, T, x->NB);
                rec_mm(x, qc[t], pc, qa[u], pa, qb[v], pb);
            }
        }
    }
}

/*
 * C[rc.., cc..] (m x n) += A[ra.., ca..] (m x k) . B[rb.., cb..] (k x n) mod p
 * on Morton-hybrid parents of sizes NC, NA, NB (each T * 2^q), by the
 * recursion of section 2.2 started on the whole (aligned) parents.  With
 * count_only set, no arithmetic is done and only the base-case calls are
 * counted.  Returns the number of base-case calls.
 */
uint64_t oracle_recursive_mm(uint32_t *C, int64_t NC, int64_t rc, int64_t cc,
                             const uint32_t *A, int64_t NA, int64_t ra, int64_t ca,
                             const uint32_t *B, int64_t NB, int64_t rb, int64_t cb,
                             int64_t m, int64_t k, int64_t n, uint32_t p, int64_t T,
                             int count_only)
{
    rec_ctx x = {C, A, B, (uint64_t)NC, (uint64_t)NA, (uint64_t)NB, (uint64_t)T, p, count_only, 0};
    if (m <= 0 || n <= 0 || k <= 0) return 0;
    blk_t C0 = {0, (uint64_t)(NC * NC)}, A0 = {0, (uint64_t)(NA * NA)}, B0 = {0, (uint64_t)(NB * NB)};
    sub_t SC = {oracle_mh_encode((uint64_t)rc, (uint64_t)cc, (uint64_t)T, (uint64_t)NC), m, n, 0, 0};
    sub_t SA = {oracle_mh_encode((uint64_t)ra, (uint64_t)ca, (uint64_t)T, (uint64_t)NA), m, k, 0, 0};
    sub_t SB = {oracle_mh_encode((uint64_t)rb, (uint64_t)cb, (uint64_t)T, (uint64_t)NB), k, n, 0, 0};
    rec_mm(&x, C0, SC, A0, SA, B0, SB);
    return x.leaves;
}

/* ------------------------------------------------------------------------ */
/* Limb digits.                                                             */
/* ------------------------------------------------------------------------ */

/*
 * Balanced base-256 digits of residue x in [0,p): the centred value
 * x' = x if x <= H else x - p, with H = 127 (256^L - 1)/255, written as
 * x' = sum_t d_t 256^t with every d_t in [-128, 127].  Digits are found one
 * at a time from the least significant: d = x' mod 256 taken in [-128,127],
 * then x' <- (x' - d) / 256.  Returns 0 if x' is not representable with L
 * digits (p > 256^L), else 1.
 */
int oracle_limb_digits(uint32_t x, uint32_t p, int L, int8_t *d)
{
    int64_t H = 0, w = 1;
    for (int t = 0; t < L; ++t) { H += 127 * w; w *= 256; }
    int64_t v = (int64_t)x <= H ? (int64_t)x : (int64_t)x - (int64_t)p;
    for (int t = 0; t < L; ++t) {
        int64_t r = ((v % 256) + 256) % 256;
        if (r > 127) r -= 256;
        d[t] = (int8_t)r;
        v = (v - r) / 256;
    }
    return v == 0;
}
