/*
 * CPU FP64 oracle for SpAMM with error control (Artemov & Rubensson,
 * "Sparse approximate matrix-matrix multiplication for density matrix
 * purification with error control").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the tests, the smoke entry point and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * Built with -O2 -ffp-contract=off -fno-fast-math: every floating-point
 * operation below is one IEEE round-to-nearest operation, in source order.
 * OpenMP is used only across independent output blocks, so results do not
 * depend on the thread count.
 *
 * Matrices are handed over as a block map: map[r*nb + c] is the index of the
 * present block (r, c) in a value array (b*b doubles per block, column-major
 * inside the block), or -1 when the block is absent (identically zero
 * quadrant of the quadtree, eq. (2)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Exact sums of squares.                                                    */
/*                                                                           */
/* The Frobenius norm used in the skip test of Algorithm 2 and the leaf      */
/* values of Algorithm 3 is read as                                          */
/*      nu(X) = sqrt_RN( RN( sum x^2 ) ),                                    */
/* the exact sum of squares rounded once to double, then a correctly rounded */
/* square root.  The exact sum is held as a big unsigned integer in units of */
/* 2^-2148 (the square of the smallest subnormal), so no bit is ever lost.   */
/* ------------------------------------------------------------------------ */

#define BIG_LIMBS 72 /* 72*64 = 4608 bits > 2148 + 2048 + 106 + carry room */

typedef struct {
    uint64_t w[BIG_LIMBS];
    int bad; /* a NaN or infinity was seen */
} big_t;

static void big_clear(big_t* a) { memset(a, 0, sizeof(*a)); }

/* a += v * 2^shift, v < 2^128 */
static void big_add_shifted(big_t* a, unsigned __int128 v, int shift) {
    int q = shift >> 6, o = shift & 63;
    uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
    uint64_t w0 = lo << o;
    uint64_t w1 = (o ? (lo >> (64 - o)) : 0) | (hi << o);
    uint64_t w2 = o ? (hi >> (64 - o)) : 0;
    uint64_t add[3] = {w0, w1, w2};
    unsigned __int128 carry = 0;
    for (int t = 0; q + t < BIG_LIMBS; ++t) {
        unsigned __int128 s = (unsigned __int128)a->w[q + t] + carry + (t < 3 ? add[t] : 0);
        a->w[q + t] = (uint64_t)s;
        carry = s >> 64;
        if (t >= 2 && carry == 0) break;
    }
}

/* Add x^2 exactly. */
static void big_add_square(big_t* a, double x) {
    if (!isfinite(x)) { a->bad = 1; return; }
    if (x == 0.0) return;
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int ex = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & ((1ull << 52) - 1);
    int e;
    if (ex == 0) { e = -1074; }            /* subnormal: x = m * 2^-1074 */
    else { m |= 1ull << 52; e = ex - 1075; } /* normal: x = m * 2^(ex-1075) */
    unsigned __int128 m2 = (unsigned __int128)m * m;
    big_add_shifted(a, m2, 2 * e + 2148);
}

/* Add a nonnegative double d exactly (d = m * 2^e, e >= -1074). */
static void big_add_double(big_t* a, double d) {
    if (!isfinite(d)) { a->bad = 1; return; }
    if (d == 0.0) return;
    uint64_t bits;
    memcpy(&bits, &d, 8);
    int ex = (int)((bits >> 52) & 0x7ff);
    uint64_t m = bits & ((1ull << 52) - 1);
    int e;
    if (ex == 0) { e = -1074; } else { m |= 1ull << 52; e = ex - 1075; }
    big_add_shifted(a, (unsigned __int128)m, e + 2148);
}

static int big_bit(const big_t* a, int i) { return (int)((a->w[i >> 6] >> (i & 63)) & 1u); }

static int big_any_below(const big_t* a, int i) { /* any set bit at index < i */
    if (i <= 0) return 0;
    int q = i >> 6, o = i & 63;
    for (int t = 0; t < q; ++t) if (a->w[t]) return 1;
    if (o && (a->w[q] & ((1ull << o) - 1))) return 1;
    return 0;
}

/* Round the exact value (units 2^-2148) to the nearest double, ties to even. */
static double big_round(const big_t* a) {
    if (a->bad) return NAN;
    int P = -1;
    for (int t = BIG_LIMBS - 1; t >= 0; --t)
        if (a->w[t]) { P = t * 64 + 63 - __builtin_clzll(a->w[t]); break; }
    if (P < 0) return 0.0;
    if (P - 2148 >= 1024) return INFINITY;
    int lsb = P - 52;
    if (lsb < 1074) lsb = 1074; /* subnormal granularity 2^-1074 */
    uint64_t M = 0;
    for (int i = P; i >= lsb; --i) M = (M << 1) | (uint64_t)big_bit(a, i);
    int rbit = lsb >= 1 ? big_bit(a, lsb - 1) : 0;
    int sticky = big_any_below(a, lsb - 1);
    if (rbit && (sticky || (M & 1u))) M += 1;
    return ldexp((double)M, lsb - 2148);
}

/* RN(sum of squares) of one block and its norm sqrt_RN of that. */
void o_block_sq(const double* v, int64_t len, double* sq, double* nu) {
    big_t acc;
    big_clear(&acc);
    for (int64_t t = 0; t < len; ++t) big_add_square(&acc, v[t]);
    double s = big_round(&acc);
    *sq = s;
    *nu = sqrt(s);
}

void o_norms(int64_t nblk, int b, const double* vals, double* sq, double* nu) {
    const int64_t bb = (int64_t)b * b;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nblk; ++k) o_block_sq(vals + k * bb, bb, sq + k, nu + k);
}

/* RN of the exact sum of nonnegative doubles. */
double o_exact_sum_nonneg(const double* v, int64_t len) {
    big_t acc;
    big_clear(&acc);
    for (int64_t t = 0; t < len; ++t) big_add_double(&acc, v[t]);
    return big_round(&acc);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3 (CSE), written as the recursion the paper gives.             */
/*                                                                           */
/* The block grid is padded to 2^L x 2^L with structurally absent blocks.   */
/* A node of the product recursion is an A-quadrant (rows ar.., cols ac..)  */
/* and a B-quadrant (rows ac.., cols bc..) of the same size.                */
/* Leaf value of candidate k (mode 0, the paper):  p if p < tau_k else 0,    */
/*   p = RN(nu(A) * nu(B)).                                                  */
/* Mode 1 (precision tiers, a bound for leaf products evaluated in a lower  */
/* precision; not in the paper): the skip threshold is the fixed tau0 and   */
/* tau_k is the low-precision limit sigma_k:                                */
/*   p < tau0 -> p;  tau0 <= p < sigma_k -> RN(c_low * p);  else 0.          */
/* Internal node (a = row half of C outer, c = column half inner):          */
/*   acc = RN(acc + RN(t*t)),  t = RN(E1 + E2), E1 from (a,0)x(0,c),         */
/*   E2 from (a,1)x(1,c);  value = sqrt_RN(acc).                             */
/* A node with either quadrant structurally empty returns zeros (the zero   */
/* test of Algorithm 3).                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nb, N, mode;
    const int32_t *mapA, *mapB;
    const double *nuA, *nuB, *tau;
    const int32_t *cntA, *cntB; /* 2D inclusive prefix counts, (nb+1)^2 */
    double tau0, c_low;
    const double* leafvals; /* optional explicit leaf values [i][k][j] (N = 1) */
    double* scratch; /* 3*N doubles per recursion depth */
} cse_ctx;

static int rect_count(const int32_t* cnt, int nb, int r0, int c0, int size) {
    int r1 = r0 + size, c1 = c0 + size;
    if (r0 >= nb || c0 >= nb) return 0;
    if (r1 > nb) r1 = nb;
    if (c1 > nb) c1 = nb;
    int W = nb + 1;
    return cnt[r1 * W + c1] - cnt[r0 * W + c1] - cnt[r1 * W + c0] + cnt[r0 * W + c0];
}

static void cse_rec(const cse_ctx* x, int ar, int ac, int bc, int size, int depth, double* out) {
    const int N = x->N;
    for (int k = 0; k < N; ++k) out[k] = 0.0;
    if (rect_count(x->cntA, x->nb, ar, ac, size) == 0 || rect_count(x->cntB, x->nb, ac, bc, size) == 0)
        return;
    if (size == 1) {
        if (x->leafvals) {
            out[0] = x->leafvals[((int64_t)ar * x->nb + ac) * x->nb + bc];
            return;
        }
        int sa = x->mapA[(int64_t)ar * x->nb + ac], sb = x->mapB[(int64_t)ac * x->nb + bc];
        double p = x->nuA[sa] * x->nuB[sb];
        for (int k = 0; k < N; ++k) {
            if (x->mode == 0) {
                if (p < x->tau[k]) out[k] = p;
            } else {
                if (p < x->tau0) out[k] = p;
                else if (p < x->tau[k]) out[k] = x->c_low * p;
            }
        }
        return;
    }
    int h = size / 2;
    double* e1 = x->scratch + (int64_t)depth * 3 * N;
    double* e2 = e1 + N;
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
            cse_rec(x, ar + a * h, ac, bc + c * h, h, depth + 1, e1);
            cse_rec(x, ar + a * h, ac + h, bc + c * h, h, depth + 1, e2);
            for (int k = 0; k < N; ++k) {
                double t = e1[k] + e2[k];
                double t2 = t * t;
                out[k] = out[k] + t2;
            }
        }
    for (int k = 0; k < N; ++k) out[k] = sqrt(out[k]);
}

static int32_t* prefix_counts(const int32_t* map, int nb) {
    int W = nb + 1;
    int32_t* cnt = (int32_t*)calloc((size_t)W * W, sizeof(int32_t));
    for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c)
            cnt[(r + 1) * W + c + 1] = cnt[r * W + c + 1] + cnt[(r + 1) * W + c] - cnt[r * W + c] +
                                       (map[(int64_t)r * nb + c] >= 0 ? 1 : 0);
    return cnt;
}

/* bound[k] for every candidate; returns 0, or -1 on bad arguments. */
int o_cse_tree(int nb, const int32_t* mapA, const double* nuA, const int32_t* mapB, const double* nuB,
               const double* tau, int N, int mode, double tau0, double c_low, double* bound) {
    if (nb < 1 || N < 1) return -1;
    int L = 0;
    while ((1 << L) < nb) ++L;
    cse_ctx x;
    x.nb = nb; x.N = N; x.mode = mode;
    x.mapA = mapA; x.mapB = mapB; x.nuA = nuA; x.nuB = nuB; x.tau = tau;
    x.tau0 = tau0; x.c_low = c_low;
    x.leafvals = NULL;
    x.cntA = prefix_counts(mapA, nb);
    x.cntB = prefix_counts(mapB, nb);
    x.scratch = (double*)malloc(sizeof(double) * 3 * (size_t)N * (L + 2));
    cse_rec(&x, 0, 0, 0, 1 << L, 0, bound);
    free(x.scratch);
    free((void*)x.cntA);
    free((void*)x.cntB);
    return 0;
}

/* The same recursion with the leaf values given explicitly
 * (leafvals[(i*nb + k)*nb + j], one candidate): the combination rule of
 * Algorithm 3 applied to an arbitrary skip pattern.                         */
int o_cse_tree_leafvals(int nb, const int32_t* mapA, const int32_t* mapB, const double* leafvals, double* bound) {
    if (nb < 1) return -1;
    int L = 0;
    while ((1 << L) < nb) ++L;
    cse_ctx x;
    memset(&x, 0, sizeof(x));
    x.nb = nb; x.N = 1; x.mapA = mapA; x.mapB = mapB; x.leafvals = leafvals;
    x.cntA = prefix_counts(mapA, nb);
    x.cntB = prefix_counts(mapB, nb);
    x.scratch = (double*)malloc(sizeof(double) * 3 * (size_t)(L + 2));
    cse_rec(&x, 0, 0, 0, 1 << L, 0, bound);
    free(x.scratch);
    free((void*)x.cntA);
    free((void*)x.cntB);
    return 0;
}

/* The two comparison bounds (used for invariants only):
 *   flat[k] = sqrt( sum_ij ( sum_{kk: p < tau_k} p )^2 )   (eq. (6) at leaf level)
 *   sum[k]  = sum over skipped pairs of p.                                      */
/* Leaf-level bounds for every candidate.  Per output (i, j) the leaf       */
/* values are summed in ascending k, one rounding per addition: s_ij.       */
/* B_sum  = RN(exact sum over outputs of s_ij),                             */
/* B_flat = sqrt_RN(RN(exact sum over outputs of RN(s_ij^2))):              */
/* exactly rounded outer sums, so the result does not depend on the order   */
/* in which the outputs are visited.                                        */
void o_cse_flat_sum(int nb, const int32_t* mapA, const double* nuA, const int32_t* mapB, const double* nuB,
                    const double* tau, int N, int mode, double tau0, double c_low, double* flat, double* sum) {
    double* colsum = (double*)malloc(sizeof(double) * N);
    big_t* accf = (big_t*)calloc((size_t)N, sizeof(big_t));
    big_t* accs = (big_t*)calloc((size_t)N, sizeof(big_t));
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            for (int k = 0; k < N; ++k) colsum[k] = 0.0;
            int any = 0;
            for (int kk = 0; kk < nb; ++kk) {
                int sa = mapA[(int64_t)i * nb + kk], sb = mapB[(int64_t)kk * nb + j];
                if (sa < 0 || sb < 0) continue;
                double p = nuA[sa] * nuB[sb];
                for (int k = 0; k < N; ++k) {
                    /* the leaf value of the CSE rule: p when skipped, c_low p
                       in the low tier (mode 1), nothing when kept exactly */
                    double v;
                    if (mode == 0) v = p < tau[k] ? p : 0.0;
                    else v = p < tau0 ? p : (p < tau[k] ? c_low * p : 0.0);
                    if (v != 0.0) { colsum[k] += v; any = 1; }
                }
            }
            if (any)
                for (int k = 0; k < N; ++k) {
                    big_add_double(&accs[k], colsum[k]);
                    big_add_double(&accf[k], colsum[k] * colsum[k]);
                }
        }
    for (int k = 0; k < N; ++k) {
        sum[k] = big_round(&accs[k]);
        flat[k] = sqrt(big_round(&accf[k]));
    }
    free(colsum);
    free(accf);
    free(accs);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (SpAMM) at the leaf level.                                    */
/* Kept set K(tau) = {(i,k,j): A_ik, B_kj present, RN(nu_A nu_B) >= tau}.    */
/* Because a leaf's norm never exceeds its ancestors' norms, skipping at     */
/* internal levels removes exactly the leaves this test removes.            */
/* sym != 0 restricts the outputs to i <= j.                                 */
/* ------------------------------------------------------------------------ */

void o_kept_counts(int nb, const int32_t* mapA, const double* nuA, const int32_t* mapB, const double* nuB,
                   double tau, int sym, int32_t* counts) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            int c = 0;
            if (!(sym && i > j))
                for (int k = 0; k < nb; ++k) {
                    int sa = mapA[(int64_t)i * nb + k], sb = mapB[(int64_t)k * nb + j];
                    if (sa < 0 || sb < 0) continue;
                    double p = nuA[sa] * nuB[sb];
                    if (p >= tau) ++c;
                }
            counts[(int64_t)i * nb + j] = c;
        }
}

/* For the outputs (oi[m], oj[m]) write their kept k, ascending, at kptr[m].. */
void o_kept_lists(int nb, const int32_t* mapA, const double* nuA, const int32_t* mapB, const double* nuB,
                  double tau, int64_t nout, const int32_t* oi, const int32_t* oj, const int64_t* kptr,
                  int32_t* klist) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < nout; ++m) {
        int64_t w = kptr[m];
        int i = oi[m], j = oj[m];
        for (int k = 0; k < nb; ++k) {
            int sa = mapA[(int64_t)i * nb + k], sb = mapB[(int64_t)k * nb + j];
            if (sa < 0 || sb < 0) continue;
            double p = nuA[sa] * nuB[sb];
            if (p >= tau) klist[w++] = k;
        }
    }
}

/* C_ij = sum over the listed k (in list order) of the textbook product
 * A_ik * B_kj: for each k, for each inner index t ascending, c += a*b.      */
void o_block_products(int b, int nb, const int32_t* mapA, const double* valsA, const int32_t* mapB,
                      const double* valsB, int64_t nout, const int32_t* oi, const int32_t* oj,
                      const int64_t* kptr, const int32_t* klist, double* out) {
    const int64_t bb = (int64_t)b * b;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t m = 0; m < nout; ++m) {
        double* C = out + m * bb;
        for (int64_t t = 0; t < bb; ++t) C[t] = 0.0;
        int i = oi[m], j = oj[m];
        for (int64_t q = kptr[m]; q < kptr[m + 1]; ++q) {
            int k = klist[q];
            const double* A = valsA + (int64_t)mapA[(int64_t)i * nb + k] * bb;
            const double* B = valsB + (int64_t)mapB[(int64_t)k * nb + j] * bb;
            for (int c = 0; c < b; ++c)
                for (int t = 0; t < b; ++t) {
                    double bv = B[(int64_t)c * b + t];
                    for (int r = 0; r < b; ++r) {
                        double prod = A[(int64_t)t * b + r] * bv;
                        C[(int64_t)c * b + r] = C[(int64_t)c * b + r] + prod;
                    }
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Exact traces used by the purification driver:                            */
/*   out[0] = RN(sum_i x_ii), out[1] = RN(sum x^2), out[2] = RN(t1 - t2)      */
/* (exact sums, one rounding each).  Blocks are (brow, bcol, vals).          */
/* ------------------------------------------------------------------------ */

static void big_sub(big_t* a, const big_t* b) { /* a -= b, requires a >= b */
    unsigned __int128 borrow = 0;
    for (int t = 0; t < BIG_LIMBS; ++t) {
        unsigned __int128 s = (unsigned __int128)a->w[t] - b->w[t] - borrow;
        a->w[t] = (uint64_t)s;
        borrow = (s >> 64) ? 1 : 0;
    }
}

static int big_cmp(const big_t* a, const big_t* b) {
    for (int t = BIG_LIMBS - 1; t >= 0; --t) {
        if (a->w[t] != b->w[t]) return a->w[t] < b->w[t] ? -1 : 1;
    }
    return 0;
}

void o_traces(int64_t nblk, int b, int64_t n, const int32_t* brow, const int32_t* bcol, const double* vals,
              double* out) {
    /* diagonal: split into positive and negative parts, each exact */
    big_t dpos, dneg, sq;
    big_clear(&dpos); big_clear(&dneg); big_clear(&sq);
    const int64_t bb = (int64_t)b * b;
    for (int64_t k = 0; k < nblk; ++k) {
        const double* v = vals + k * bb;
        for (int64_t t = 0; t < bb; ++t) big_add_square(&sq, v[t]);
        if (brow[k] == bcol[k])
            for (int r = 0; r < b; ++r) {
                if ((int64_t)brow[k] * b + r >= n) break;
                double d = v[(int64_t)r * b + r];
                if (d >= 0) big_add_double(&dpos, d); else big_add_double(&dneg, -d);
            }
    }
    /* t1 = dpos - dneg; each value is scaled by 2^2148 in dpos/dneg, while
       squares use the same unit, so the three can be combined directly. */
    big_t t1 = dpos, e = dpos, tmp;
    int t1neg = 0;
    if (big_cmp(&dpos, &dneg) >= 0) big_sub(&t1, &dneg);
    else { t1 = dneg; big_sub(&t1, &dpos); t1neg = 1; }
    double t1d = big_round(&t1);
    out[0] = t1neg ? -t1d : t1d;
    out[1] = big_round(&sq);
    /* e = dpos - dneg - sq */
    tmp = dneg;
    /* tmp = dneg + sq */
    {
        unsigned __int128 carry = 0;
        for (int t = 0; t < BIG_LIMBS; ++t) {
            unsigned __int128 s = (unsigned __int128)tmp.w[t] + sq.w[t] + carry;
            tmp.w[t] = (uint64_t)s;
            carry = s >> 64;
        }
    }
    if (big_cmp(&e, &tmp) >= 0) { big_sub(&e, &tmp); out[2] = big_round(&e); }
    else { big_t f = tmp; big_sub(&f, &e); out[2] = -big_round(&f); }
    if (dpos.bad || dneg.bad || sq.bad) { out[0] = out[1] = out[2] = NAN; }
}

/* Gerschgorin discs: for each row r < n, radius = RN(exact sum_{c != r} |f_rc|),
 * centre f_rr.  out[0] = min(centre - radius), out[1] = max(centre + radius). */
void o_gerschgorin(int64_t nblk, int b, int64_t n, const int32_t* brow, const int32_t* bcol, const double* vals,
                   double* out) {
    int64_t nb = (n + b - 1) / b;
    big_t* rad = (big_t*)calloc((size_t)(nb * b), sizeof(big_t));
    double* cen = (double*)calloc((size_t)(nb * b), sizeof(double));
    const int64_t bb = (int64_t)b * b;
    for (int64_t k = 0; k < nblk; ++k) {
        const double* v = vals + k * bb;
        for (int c = 0; c < b; ++c)
            for (int r = 0; r < b; ++r) {
                int64_t gi = (int64_t)brow[k] * b + r, gj = (int64_t)bcol[k] * b + c;
                double x = v[(int64_t)c * b + r];
                if (gi >= n || gj >= n) continue;
                if (gi == gj) cen[gi] = x;
                else big_add_double(&rad[gi], fabs(x));
            }
    }
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double R = big_round(&rad[i]);
        double a = cen[i] - R, z = cen[i] + R;
        if (a < lo) lo = a;
        if (z > hi) hi = z;
    }
    out[0] = lo;
    out[1] = hi;
    free(rad);
    free(cen);
}
