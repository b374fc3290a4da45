/*
 * QHap CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 reference of what the phasing hot path computes, written
 * from the paper's Methods section.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header or table with the GPU library.
 *
 * Graphs are held as CSR over structural pairs (i != j), columns ascending,
 * values in FP64.  Spin / momentum state is [n][R], replica index fastest.
 *
 * Readings of the paper taken here where it is silent or ambiguous:
 *  - The read graph keeps every co-covered pair as a structural edge, even when
 *    its weight is 0 (such an edge adds 0 to any cut).
 *  - Signed read weights J_ab = sum_j M_aj M_bj ("agree minus disagree") are
 *    offered beside the paper's conflict count A_ab = sum_j [M_aj M_bj = -1].
 *  - SNP weights: observations with Phred Q <= 3 are dropped (q <= 0.5 makes
 *    the log-likelihood ratio vanish or flip sign; Q = 0 divides by zero);
 *    |S_i| counts the kept observations of fragment i, before the linkage-depth
 *    truncation; each SNP links to the floor(k(|S_i|-1)/10) nearest downstream
 *    SNPs of the fragment; the Pore-C factor alpha_i multiplies fragment i's terms.
 *  - bSB (ballistic simulated bifurcation, cited by the paper): symplectic Euler
 *    with y updated first, then x, then the inelastic walls at |x| = 1.
 *  - Initial x, y: i.i.d. U(-0.1, 0.1) from SplitMix64 (counter-based).
 *  - sgn(0) = +1.
 *  - Greedy single-flip rounds flip an independent set of strictly improving
 *    vertices: i flips when g_i > eps and g_i beats every improving neighbour
 *    (ties broken toward the lower index).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Eq. (1), Methods "Matrix construction": ternary encoding against H1.        */
/* Every observation carries one of the two alleles, so M is +1 where the      */
/* observed allele equals H1[j] and -1 where it equals H2[j] = 1 - H1[j].      */
/* ------------------------------------------------------------------------- */
void or_encode(int64_t nobs, const int32_t *snp, const uint8_t *allele,
               const uint8_t *init_h1, int8_t *M) {
    for (int64_t t = 0; t < nobs; ++t) {
        uint8_t h1 = init_h1[snp[t]];
        uint8_t h2 = (uint8_t)(1 - h1);
        if (allele[t] == h1) M[t] = 1;
        else if (allele[t] == h2) M[t] = -1;
        else M[t] = 0;
    }
}

/* Per-SNP coverage lists (fragment id and observation index), fragments ascending. */
static int build_coverage(int64_t n_snp, int64_t n_frag, const int64_t *frag_ptr,
                          const int32_t *snp, const uint8_t *keep,
                          int64_t **cov_ptr_out, int64_t **cov_frag_out, int64_t **cov_obs_out) {
    int64_t nobs = frag_ptr[n_frag];
    int64_t *cov_ptr = calloc((size_t)n_snp + 1, sizeof(int64_t));
    if (!cov_ptr) return OR_ENOMEM;
    for (int64_t t = 0; t < nobs; ++t)
        if (!keep || keep[t]) cov_ptr[snp[t] + 1]++;
    for (int64_t j = 0; j < n_snp; ++j) cov_ptr[j + 1] += cov_ptr[j];
    int64_t total = cov_ptr[n_snp];
    int64_t *cf = malloc((size_t)(total ? total : 1) * sizeof(int64_t));
    int64_t *co = malloc((size_t)(total ? total : 1) * sizeof(int64_t));
    int64_t *fill = malloc((size_t)(n_snp ? n_snp : 1) * sizeof(int64_t));
    if (!cf || !co || !fill) { free(cov_ptr); free(cf); free(co); free(fill); return OR_ENOMEM; }
    memcpy(fill, cov_ptr, (size_t)n_snp * sizeof(int64_t));
    for (int64_t f = 0; f < n_frag; ++f)
        for (int64_t t = frag_ptr[f]; t < frag_ptr[f + 1]; ++t) {
            if (keep && !keep[t]) continue;
            int64_t s = fill[snp[t]]++;
            cf[s] = f;
            co[s] = t;
        }
    free(fill);
    *cov_ptr_out = cov_ptr;
    *cov_frag_out = cf;
    *cov_obs_out = co;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Eqs. (2)-(3), Methods "Max-Cut graph construction" (read-based):            */
/*   conflict (kind 0): w_ab = sum_j 1[M_aj * M_bj = -1]                       */
/*   signed   (kind 1): J_ab = sum_j M_aj * M_bj                               */
/* Output: dense n_frag x n_frag int64 weights and int32 co-coverage counts.    */
/* The sum runs column by column over the fragments covering SNP j.             */
/* ------------------------------------------------------------------------- */
int or_read_graph_dense(int kind, int64_t n_snp, int64_t n_frag, const int64_t *frag_ptr,
                        const int32_t *snp, const int8_t *M, int64_t *W, int32_t *C) {
    int64_t *cov_ptr, *cov_frag, *cov_obs;
    int rc = build_coverage(n_snp, n_frag, frag_ptr, snp, NULL, &cov_ptr, &cov_frag, &cov_obs);
    if (rc) return rc;
    memset(W, 0, (size_t)(n_frag * n_frag) * sizeof(int64_t));
    memset(C, 0, (size_t)(n_frag * n_frag) * sizeof(int32_t));
    for (int64_t j = 0; j < n_snp; ++j) {
        for (int64_t p = cov_ptr[j]; p < cov_ptr[j + 1]; ++p) {
            for (int64_t q = cov_ptr[j]; q < cov_ptr[j + 1]; ++q) {
                int64_t a = cov_frag[p], b = cov_frag[q];
                if (a == b) continue;
                int prod = (int)M[cov_obs[p]] * (int)M[cov_obs[q]];
                if (kind == 0) W[a * n_frag + b] += (prod == -1) ? 1 : 0;
                else W[a * n_frag + b] += prod;
                C[a * n_frag + b] += 1;
            }
        }
    }
    free(cov_ptr); free(cov_frag); free(cov_obs);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Eqs. (9)-(14), Methods "SNP-based method": quality-weighted log-likelihood   */
/* edge weights, with the linkage depth of "SNP linkage depth analysis" and    */
/* the Pore-C factor alpha of "Pore-C data support".                            */
/* ------------------------------------------------------------------------- */

/* Eq. (9): confidence from a Phred score. */
static double phred_confidence(int Q) { return 1.0 - pow(10.0, -(double)Q / 10.0); }

/* Eqs. (11)-(13): l = sgn(W_iu W_iv) * log10(P_cis / P_trans). */
static double llr_term(int8_t Mu, int8_t Mv, int Qu, int Qv) {
    double qu = phred_confidence(Qu), qv = phred_confidence(Qv);
    double p_cis = qu * qv + (1.0 - qu) * (1.0 - qv);
    double p_trans = qu * (1.0 - qv) + (1.0 - qu) * qv;
    double sgn = ((int)Mu * (int)Mv > 0) ? 1.0 : -1.0;
    return sgn * log10(p_cis / p_trans);
}

typedef struct {
    int64_t *kept_ptr;   /* per fragment: range in kept_obs */
    int64_t *kept_obs;   /* observation indices with Q > 3, fragment order */
    int64_t *obs_rank;   /* observation -> rank inside its fragment's kept list, -1 if dropped */
} kept_lists;

static int build_kept(int64_t n_frag, const int64_t *frag_ptr, const uint8_t *phred, kept_lists *kl) {
    int64_t nobs = frag_ptr[n_frag];
    kl->kept_ptr = calloc((size_t)n_frag + 1, sizeof(int64_t));
    kl->kept_obs = malloc((size_t)(nobs ? nobs : 1) * sizeof(int64_t));
    kl->obs_rank = malloc((size_t)(nobs ? nobs : 1) * sizeof(int64_t));
    if (!kl->kept_ptr || !kl->kept_obs || !kl->obs_rank) return OR_ENOMEM;
    int64_t k = 0;
    for (int64_t f = 0; f < n_frag; ++f) {
        kl->kept_ptr[f] = k;
        int64_t r = 0;
        for (int64_t t = frag_ptr[f]; t < frag_ptr[f + 1]; ++t) {
            if (phred[t] > 3) { kl->kept_obs[k++] = t; kl->obs_rank[t] = r++; }
            else kl->obs_rank[t] = -1;
        }
    }
    kl->kept_ptr[n_frag] = k;
    return OR_OK;
}

static void free_kept(kept_lists *kl) { free(kl->kept_ptr); free(kl->kept_obs); free(kl->obs_rank); }

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Structure pass: row_ptr[n_snp+1] and the number of structural entries.
 * col may be NULL (count only) or receive the ascending column lists. */
int or_snp_graph_structure(int64_t n_snp, int64_t n_frag, const int64_t *frag_ptr,
                           const int32_t *snp, const uint8_t *phred, int linkage_k,
                           int64_t *row_ptr, int32_t *col) {
    kept_lists kl;
    if (build_kept(n_frag, frag_ptr, phred, &kl)) return OR_ENOMEM;
    uint8_t *keep = malloc((size_t)(frag_ptr[n_frag] ? frag_ptr[n_frag] : 1));
    for (int64_t t = 0; t < frag_ptr[n_frag]; ++t) keep[t] = phred[t] > 3;
    int64_t *cov_ptr, *cov_frag, *cov_obs;
    int rc = build_coverage(n_snp, n_frag, frag_ptr, snp, keep, &cov_ptr, &cov_frag, &cov_obs);
    if (rc) { free(keep); free_kept(&kl); return rc; }
    int fail = 0;
    row_ptr[0] = 0;
    /* count pass (serial prefix below) */
    int64_t *cnt = calloc((size_t)n_snp, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < n_snp; ++u) {
        int64_t cap = 0;
        for (int64_t p = cov_ptr[u]; p < cov_ptr[u + 1]; ++p) {
            int64_t f = cov_frag[p];
            int64_t ns = kl.kept_ptr[f + 1] - kl.kept_ptr[f];
            cap += 2 * ((int64_t)linkage_k * (ns - 1) / 10) + 1;
        }
        int32_t *tmp = malloc((size_t)(cap ? cap : 1) * sizeof(int32_t));
        if (!tmp) { fail = 1; continue; }
        int64_t m = 0;
        for (int64_t p = cov_ptr[u]; p < cov_ptr[u + 1]; ++p) {
            int64_t f = cov_frag[p];
            int64_t base = kl.kept_ptr[f];
            int64_t ns = kl.kept_ptr[f + 1] - base;
            if (ns < 2) continue;
            int64_t L = (int64_t)linkage_k * (ns - 1) / 10;
            int64_t a = kl.obs_rank[cov_obs[p]];
            for (int64_t b = a - L; b <= a + L; ++b) {
                if (b < 0 || b >= ns || b == a) continue;
                tmp[m++] = snp[kl.kept_obs[base + b]];
            }
        }
        qsort(tmp, (size_t)m, sizeof(int32_t), cmp_i32);
        int64_t uniq = 0;
        for (int64_t t = 0; t < m; ++t)
            if (t == 0 || tmp[t] != tmp[t - 1]) tmp[uniq++] = tmp[t];
        cnt[u] = uniq;
        if (col && row_ptr) {
            /* second call: row_ptr already filled by the first call */
            memcpy(col + row_ptr[u], tmp, (size_t)uniq * sizeof(int32_t));
        }
        free(tmp);
    }
    if (!col) {
        for (int64_t u = 0; u < n_snp; ++u) row_ptr[u + 1] = row_ptr[u] + cnt[u];
    }
    free(cnt); free(keep); free(cov_ptr); free(cov_frag); free(cov_obs); free_kept(&kl);
    return fail ? OR_ENOMEM : OR_OK;
}

static int64_t find_col(const int32_t *col, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Value pass, Eq. (14): w_uv = - sum_{i in F_uv} alpha_i * l_uv^(i) / (|S_i| - 1).
 * Each row sums its fragments in ascending fragment order. */
int or_snp_graph_values(int64_t n_snp, int64_t n_frag, const int64_t *frag_ptr,
                        const int32_t *snp, const int8_t *M, const uint8_t *phred,
                        const double *alpha, int linkage_k,
                        const int64_t *row_ptr, const int32_t *col, double *val) {
    kept_lists kl;
    if (build_kept(n_frag, frag_ptr, phred, &kl)) return OR_ENOMEM;
    uint8_t *keep = malloc((size_t)(frag_ptr[n_frag] ? frag_ptr[n_frag] : 1));
    for (int64_t t = 0; t < frag_ptr[n_frag]; ++t) keep[t] = phred[t] > 3;
    int64_t *cov_ptr, *cov_frag, *cov_obs;
    int rc = build_coverage(n_snp, n_frag, frag_ptr, snp, keep, &cov_ptr, &cov_frag, &cov_obs);
    if (rc) { free(keep); free_kept(&kl); return rc; }
    memset(val, 0, (size_t)row_ptr[n_snp] * sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < n_snp; ++u) {
        for (int64_t p = cov_ptr[u]; p < cov_ptr[u + 1]; ++p) {
            int64_t f = cov_frag[p];
            int64_t base = kl.kept_ptr[f];
            int64_t ns = kl.kept_ptr[f + 1] - base;
            if (ns < 2) continue;
            int64_t L = (int64_t)linkage_k * (ns - 1) / 10;
            int64_t tu = cov_obs[p];
            int64_t a = kl.obs_rank[tu];
            double af = alpha ? alpha[f] : 1.0;
            for (int64_t b = a - L; b <= a + L; ++b) {
                if (b < 0 || b >= ns || b == a) continue;
                int64_t tv = kl.kept_obs[base + b];
                int32_t v = snp[tv];
                double l = llr_term(M[tu], M[tv], phred[tu], phred[tv]);
                int64_t slot = find_col(col, row_ptr[u], row_ptr[u + 1], v);
                val[slot] -= af * l / (double)(ns - 1);
            }
        }
    }
    free(keep); free(cov_ptr); free(cov_frag); free(cov_obs); free_kept(&kl);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Connected components by breadth-first search (Methods, read- and SNP-based */
/* graph construction).  Components are numbered in the order of their lowest */
/* vertex; single-vertex components get label -1 (excluded from phasing).      */
/* ------------------------------------------------------------------------- */
int64_t or_components(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t *comp) {
    int64_t *queue = malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) comp[i] = -2;
    int32_t next = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (comp[s] != -2) continue;
        if (row_ptr[s + 1] == row_ptr[s]) { comp[s] = -1; continue; }
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        comp[s] = next;
        while (head < tail) {
            int64_t v = queue[head++];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t w = col[e];
                if (comp[w] == -2) { comp[w] = next; queue[tail++] = w; }
            }
        }
        next++;
    }
    free(queue);
    return next;
}

/* ------------------------------------------------------------------------- */
/* Coupling scale of ballistic SB: c0 = 0.5 / (sigma_J * sqrt(N)) with         */
/* sigma_J^2 = sum_{i != j} J_ij^2 / (N (N - 1)).                              */
/* ------------------------------------------------------------------------- */
double or_c0(int64_t n, const int64_t *row_ptr, const double *val) {
    double ss = 0.0;
    for (int64_t e = 0; e < row_ptr[n]; ++e) ss += val[e] * val[e];
    if (ss <= 0.0 || n < 2) return 0.0;
    double sigma = sqrt(ss / ((double)n * (double)(n - 1)));
    return 0.5 / (sigma * sqrt((double)n));
}

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the k-th output of the       */
/* stream seeded with s is mix(s + (k + 1) * 0x9E3779B97F4A7C15).               */
/* ------------------------------------------------------------------------- */
uint64_t or_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* x0[i][r], y0[i][r] ~ U(-0.1, 0.1): draw k = 2 (r n + i) + {0: x, 1: y}. */
void or_init(uint64_t seed, int64_t n, int R, double *x, double *y) {
    for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < R; ++r) {
            uint64_t c = 2 * ((uint64_t)r * (uint64_t)n + (uint64_t)i);
            double ux = (double)(or_splitmix64(seed, c) >> 11) * 0x1.0p-53;
            double uy = (double)(or_splitmix64(seed, c + 1) >> 11) * 0x1.0p-53;
            x[i * R + r] = 0.2 * ux - 0.1;
            y[i * R + r] = 0.2 * uy - 0.1;
        }
}

/* ------------------------------------------------------------------------- */
/* Ballistic simulated bifurcation (Methods "SB algorithm solution"):           */
/*   y_i <- y_i + [-(a0 - p_k) x_i + c0 sum_j J_ij x_j] dt                      */
/*   x_i <- x_i + a0 y_i dt                                                     */
/*   |x_i| > 1  =>  x_i <- sgn(x_i), y_i <- 0                                   */
/* for k in [k_begin, k_end), all R replicas side by side.  discrete = 1 gives  */
/* the discrete variant of the same family (dSB): the coupling term uses        */
/* sgn(x_j) (sgn(0) = +1) in place of x_j; everything else is unchanged.        */
/* field (NULL = none) is the deformation term h of the adaptive strategy       */
/* (Methods, SNP "SB algorithm solution"): a per-vertex field that joins the    */
/* coupling, c0 (sum_j J_ij x_j + h_i), as the field of an Ising Hamiltonian    */
/* -1/2 x'Jx - h'x does in the bifurcation equations.                           */
/* ------------------------------------------------------------------------- */
void or_sb_run(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
               int R, int64_t k_begin, int64_t k_end, const double *pump,
               double dt, double c0, double a0, double *x, double *y, int discrete, const double *field) {
    double *xnew = malloc((size_t)(n * R) * sizeof(double));
    double *z = malloc((size_t)(n * R) * sizeof(double));
    for (int64_t k = k_begin; k < k_end; ++k) {
        double p = pump[k];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double *zi = z + i * R;
            for (int r = 0; r < R; ++r) zi[r] = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                double J = val[e];
                const double *xj = x + (int64_t)col[e] * R;
                if (discrete)
                    for (int r = 0; r < R; ++r) zi[r] += J * (xj[r] >= 0.0 ? 1.0 : -1.0);
                else
                    for (int r = 0; r < R; ++r) zi[r] += J * xj[r];
            }
            const double hi = field ? field[i] : 0.0;
            for (int r = 0; r < R; ++r) {
                double yi = y[i * R + r] + (-(a0 - p) * x[i * R + r] + c0 * (zi[r] + hi)) * dt;
                double xi = x[i * R + r] + a0 * yi * dt;
                if (fabs(xi) > 1.0) { xi = xi > 0 ? 1.0 : -1.0; yi = 0.0; }
                y[i * R + r] = yi;
                xnew[i * R + r] = xi;
            }
        }
        memcpy(x, xnew, (size_t)(n * R) * sizeof(double));
    }
    free(xnew); free(z);
}

void or_bsb_run(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                int R, int64_t k_begin, int64_t k_end, const double *pump,
                double dt, double c0, double a0, double *x, double *y) {
    or_sb_run(n, row_ptr, col, val, R, k_begin, k_end, pump, dt, c0, a0, x, y, 0, NULL);
}

/* Linear pump 0 -> 1 with both ends included. */
void or_pump_linear(int64_t steps, double *pump) {
    for (int64_t k = 0; k < steps; ++k)
        pump[k] = steps > 1 ? (double)k / (double)(steps - 1) : 0.0;
}

/* Sign readout s = sgn(x), sgn(0) = +1. */
void or_signs(int64_t count, const double *x, int8_t *s) {
    for (int64_t t = 0; t < count; ++t) s[t] = x[t] >= 0.0 ? 1 : -1;
}

/* ------------------------------------------------------------------------- */
/* Eqs. (4)-(6): A = -J; cut(s) = 1/4 sum_{a,b} A_ab (1 - s_a s_b), per        */
/* replica and per component (rows of label -1 are skipped).                   */
/* cut[r * n_comp + c].                                                         */
/* ------------------------------------------------------------------------- */
void or_cuts(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
             const int32_t *comp, int64_t n_comp, int R, const int8_t *s, double *cut) {
    for (int64_t t = 0; t < (int64_t)R * n_comp; ++t) cut[t] = 0.0;
    for (int r = 0; r < R; ++r)
        for (int64_t a = 0; a < n; ++a) {
            if (comp[a] < 0) continue;
            double acc = 0.0;
            for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e) {
                double A = -val[e];
                int sa = s[a * R + r], sb = s[(int64_t)col[e] * R + r];
                acc += A * (1.0 - (double)(sa * sb));
            }
            cut[(int64_t)r * n_comp + comp[a]] += 0.25 * acc;
        }
}

/* Eq. (5): E(s) = -1/2 s^T J s for each replica. */
void or_energy(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
               int R, const int8_t *s, double *E) {
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        for (int64_t a = 0; a < n; ++a)
            for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e)
                acc += (double)s[a * R + r] * val[e] * (double)s[(int64_t)col[e] * R + r];
        E[r] = -0.5 * acc;
    }
}

/* Best replica per component (ties -> lowest r), oriented so that the
 * component's lowest-index vertex reads +1; singletons read +1. */
void or_select(int64_t n, const int32_t *comp, int64_t n_comp, int R, const int8_t *s,
               const double *cut, int8_t *best, int32_t *best_r) {
    for (int64_t c = 0; c < n_comp; ++c) {
        int br = 0;
        for (int r = 1; r < R; ++r)
            if (cut[(int64_t)r * n_comp + c] > cut[(int64_t)br * n_comp + c]) br = r;
        best_r[c] = br;
    }
    int8_t *orient = malloc((size_t)(n_comp ? n_comp : 1));
    uint8_t *seen = calloc((size_t)(n_comp ? n_comp : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = comp[i];
        if (c < 0) { best[i] = 1; continue; }
        int8_t v = s[i * R + best_r[c]];
        if (!seen[c]) { seen[c] = 1; orient[c] = v; }
        best[i] = (int8_t)(v * orient[c]);
    }
    free(orient); free(seen);
}

/* ------------------------------------------------------------------------- */
/* Greedy single-flip rounds on one spin vector.  Gain of flipping i:           */
/*   g_i = s_i sum_j A_ij s_j = -s_i sum_j J_ij s_j.                            */
/* A round flips every i with g_i > eps that beats each neighbour j (J_ij != 0) */
/* with g_j > eps (larger gain, or equal gain and lower index).  Returns the    */
/* number of rounds that flipped something.                                     */
/* ------------------------------------------------------------------------- */
int64_t or_greedy(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                  double eps, int64_t max_rounds, int8_t *s) {
    double *g = malloc((size_t)(n ? n : 1) * sizeof(double));
    uint8_t *flip = malloc((size_t)(n ? n : 1));
    int64_t rounds = 0;
    while (rounds < max_rounds) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                acc += -val[e] * (double)s[col[e]];
            g[i] = (double)s[i] * acc;
        }
        int64_t nflip = 0;
        for (int64_t i = 0; i < n; ++i) {
            flip[i] = 0;
            if (!(g[i] > eps)) continue;
            int win = 1;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1] && win; ++e) {
                int32_t j = col[e];
                if (val[e] == 0.0 || !(g[j] > eps)) continue;
                if (g[j] > g[i] || (g[j] == g[i] && j < i)) win = 0;
            }
            if (win) { flip[i] = 1; nflip++; }
        }
        if (nflip == 0) break;
        for (int64_t i = 0; i < n; ++i)
            if (flip[i]) s[i] = (int8_t)-s[i];
        rounds++;
    }
    free(g); free(flip);
    return rounds;
}

/* ------------------------------------------------------------------------- */
/* Eqs. (7)-(8) and the hierarchical rule of "Consistency processing":          */
/* read-based consensus per SNP.  s_frag[f] = +1 puts fragment f in S1.         */
/* Fragments with comp_frag[f] < 0 (single-fragment components) do not vote.   */
/* h1[j]: allele (0/1) of output haplotype 1 (= subset S1), -1 if filtered.     */
/* block[j]: component of the fragments covering j, -1 if none.                 */
/* ------------------------------------------------------------------------- */
void or_phase_vote(int64_t n_snp, int64_t n_frag, const int64_t *frag_ptr, const int32_t *snp,
                   const int8_t *M, const int8_t *s_frag, const int32_t *comp_frag,
                   const uint8_t *init_h1, int8_t *h1, int32_t *block) {
    int64_t *c1p = calloc((size_t)n_snp, sizeof(int64_t)), *c1m = calloc((size_t)n_snp, sizeof(int64_t));
    int64_t *c2p = calloc((size_t)n_snp, sizeof(int64_t)), *c2m = calloc((size_t)n_snp, sizeof(int64_t));
    for (int64_t j = 0; j < n_snp; ++j) block[j] = -1;
    for (int64_t f = 0; f < n_frag; ++f) {
        if (comp_frag[f] < 0) continue;
        for (int64_t t = frag_ptr[f]; t < frag_ptr[f + 1]; ++t) {
            int32_t j = snp[t];
            block[j] = comp_frag[f];
            if (s_frag[f] > 0) { if (M[t] == 1) c1p[j]++; else if (M[t] == -1) c1m[j]++; }
            else { if (M[t] == 1) c2p[j]++; else if (M[t] == -1) c2m[j]++; }
        }
    }
    for (int64_t j = 0; j < n_snp; ++j) {
        uint8_t H1 = init_h1[j], H2 = (uint8_t)(1 - init_h1[j]);
        int64_t d1 = c1p[j] - c1m[j], d2 = c2p[j] - c2m[j];
        /* filters: no coverage in both subsets, or equal support in both subsets */
        if ((c1p[j] + c1m[j] == 0 && c2p[j] + c2m[j] == 0) || (d1 == 0 && d2 == 0)) {
            h1[j] = -1;
            continue;
        }
        int maj1 = (d1 > 0) - (d1 < 0), maj2 = (d2 > 0) - (d2 < 0);
        if (maj1 != 0 && maj2 != 0 && maj1 == maj2) {
            /* concordant majorities: the larger differential keeps its allele,
             * ties go to S1 */
            int64_t a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2;
            if (a1 >= a2) h1[j] = (int8_t)(maj1 > 0 ? H1 : H2);
            else h1[j] = (int8_t)(maj2 > 0 ? H2 : H1);  /* S1 takes the complement */
        } else if (maj1 != 0 && maj2 != 0) {
            /* opposing majorities: the +1 subset takes H1[j], the -1 subset H2[j] */
            h1[j] = (int8_t)(maj1 > 0 ? H1 : H2);
        } else if (maj1 != 0) {
            /* only S1 has a majority: it decides */
            h1[j] = (int8_t)(maj1 > 0 ? H1 : H2);
        } else {
            /* only S2 has a majority: S1 takes the complement */
            h1[j] = (int8_t)(maj2 > 0 ? H2 : H1);
        }
    }
    free(c1p); free(c1m); free(c2p); free(c2m);
}

/* ------------------------------------------------------------------------- */
/* Eqs. (16)-(17), one refinement round: per component, S_min is the smaller   */
/* subset (equal sizes -> the s = -1 subset); C(u) = 1[u in S_min]; H1'/H2'    */
/* swap where C(u) is odd.                                                      */
/* ------------------------------------------------------------------------- */
void or_phase_parity(int64_t n, const int32_t *comp, int64_t n_comp, const int8_t *s,
                     const uint8_t *init_h1, int8_t *h1, int32_t *block) {
    int64_t *plus = calloc((size_t)(n_comp ? n_comp : 1), sizeof(int64_t));
    int64_t *minus = calloc((size_t)(n_comp ? n_comp : 1), sizeof(int64_t));
    for (int64_t u = 0; u < n; ++u) {
        if (comp[u] < 0) continue;
        if (s[u] > 0) plus[comp[u]]++; else minus[comp[u]]++;
    }
    for (int64_t u = 0; u < n; ++u) {
        int32_t c = comp[u];
        if (c < 0) { h1[u] = -1; block[u] = -1; continue; }
        int8_t smin = plus[c] < minus[c] ? 1 : -1;
        int C = s[u] == smin ? 1 : 0;
        h1[u] = (int8_t)((C % 2 == 0) ? init_h1[u] : 1 - init_h1[u]);
        block[u] = c;
    }
    free(plus); free(minus);
}

/* Eq. (15): flip the sign of every edge that crosses the partition. */
void or_flip_crossing(int64_t n, const int64_t *row_ptr, const int32_t *col, double *val,
                      const int8_t *s) {
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (s[u] != s[col[e]]) val[e] = -val[e];
}
