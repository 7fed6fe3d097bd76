/*
 * bpmf_oracle.c -- plain, slow, FP64 CPU reference of the BPMF Gibbs sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header or constant table with the
 * HIP library: every routine below is written out from the mathematics.
 *
 * What it follows (Vander Aa, Chakroun, Haber, "Distributed Bayesian
 * Probabilistic Matrix Factorization", 2017):
 *   - Sec. I: R (M x N) ~ U V^T with U: M x K (users), V: N x K (movies).
 *   - Sec. II, Algorithm 1: one sampling iteration = hyper draw of the movie
 *     prior from V, update of every movie, hyper draw of the user prior from
 *     U, update of every user, then prediction of every test point and RMSE.
 *   - Sec. II: each item update is a handful of K x K matrix/vector
 *     operations plus one K x K "inversion"; here that inversion is a
 *     Cholesky factorisation followed by two triangular solves.
 *   - The paper defers the model to Salakhutdinov & Mnih's BPMF: Gaussian
 *     likelihood with precision alpha, Gaussian row priors N(mu, Lambda^-1),
 *     Normal-Wishart hyperpriors.  The conjugate conditionals used below are
 *     the standard ones (derived, not quoted):
 *       row i:  P = Lambda + alpha * sum_j y_j y_j^T,
 *               b = Lambda mu + alpha * sum_j r'_ij y_j,
 *               x ~ N(P^-1 b, P^-1)  drawn as  x = L^-T (L^-1 b + z), P = L L^T.
 *       hyper:  beta* = beta0 + n, nu* = nu0 + n,
 *               mu* = (beta0 mu0 + n xbar) / beta*,
 *               W*^-1 = W0^-1 + S + beta0 n / beta* (xbar - mu0)(xbar - mu0)^T,
 *               Lambda ~ Wishart(W*, nu*)  (Bartlett decomposition),
 *               mu ~ N(mu*, (beta* Lambda)^-1).
 *
 * Noise.  Every random number is a deterministic function of
 * (seed, counter) through Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * turned into normals by the Box-Muller transform and into chi-square
 * variates by Marsaglia & Tsang's gamma method (ACM TOMS 26(3), 2000).
 *   row noise   : counter (row, t, stream<<24 | block, 0), 4 normals per block
 *   hyper chi2  : counter (k,   t, stream<<24 | 0, attempt)
 *   hyper lower : counter (blk, t, stream<<24 | 1, 0)
 *   hyper mu    : counter (blk, t, stream<<24 | 2, 0)
 *   fold-in     : counter (lo32(req), s, stream<<24 | block, hi32(req))
 *   key         : (lo32(seed), hi32(seed))
 *
 * All arithmetic is double precision, every sum runs sequentially in stored
 * order, and rows of one side are independent, so results do not depend on
 * the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of the Philox S-box with two 32x32->64 bit      */
/* multiplications; the key is bumped by the Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                         uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Map a 32-bit word to the open interval (0, 1): (x + 1/2) * 2^-32. */
static double uniform01(uint32_t x)
{
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

/* Box-Muller on one block: (u0,u1) -> (z0,z1), (u2,u3) -> (z2,z3). */
static void box_muller4(const uint32_t w[4], double z[4])
{
    double u0 = uniform01(w[0]), u1 = uniform01(w[1]);
    double u2 = uniform01(w[2]), u3 = uniform01(w[3]);
    double ra = sqrt(-2.0 * log(u0));
    double rb = sqrt(-2.0 * log(u2));
    z[0] = ra * cos(ORC_TWO_PI * u1);
    z[1] = ra * sin(ORC_TWO_PI * u1);
    z[2] = rb * cos(ORC_TWO_PI * u3);
    z[3] = rb * sin(ORC_TWO_PI * u3);
}

/* n standard normals from blocks (c0, c1, stream<<24 | b, c3), b = 0,1,...;
 * normal k comes from block k/4, lane k%4; unused lanes are discarded.      */
void orc_normals(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t stream,
                 uint32_t c3, int n, double *z)
{
    for (int b = 0; 4 * b < n; ++b) {
        uint32_t w[4];
        double g[4];
        philox_block(seed, c0, c1, (stream << 24) | (uint32_t)b, c3, w);
        box_muller4(w, g);
        for (int l = 0; l < 4 && 4 * b + l < n; ++l) z[4 * b + l] = g[l];
    }
}

/* Chi-square with `dof` degrees of freedom = 2 * Gamma(dof/2, 1), Gamma by
 * Marsaglia-Tsang (shape a >= 1): d = a - 1/3, c = 1/sqrt(9d); propose
 * v = (1 + c x)^3 with x ~ N(0,1); accept when v > 0 and
 * log(u) < x^2/2 + d - d v + d log v.  Attempt j uses one Philox block with
 * counter (index, t, stream<<24 | 0, j): x from the cosine branch of (w0,w1),
 * u = uniform(w2).                                                           */
double orc_chi2(uint64_t seed, uint32_t stream, uint32_t t, uint32_t index,
                double dof, int32_t *attempts_out)
{
    double a = 0.5 * dof;
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t attempt = 0;; ++attempt) {
        uint32_t w[4];
        philox_block(seed, index, t, (stream << 24) | 0u, attempt, w);
        double x = sqrt(-2.0 * log(uniform01(w[0]))) * cos(ORC_TWO_PI * uniform01(w[1]));
        double u = uniform01(w[2]);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (log(u) < 0.5 * x * x + d - d * v + d * log(v)) {
            if (attempts_out) *attempts_out = (int32_t)attempt + 1;
            return 2.0 * d * v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra on row-major n x n arrays.                          */
/* ------------------------------------------------------------------------ */

/* In-place Cholesky A = L L^T (lower, positive diagonal; the strict upper
 * triangle is zeroed).  Returns 0, or -1 when a pivot is not positive.     */
int orc_cholesky(int n, double *A)
{
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return -1;
        double djj = sqrt(s);
        A[j * n + j] = djj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / djj;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return 0;
}

/* Solve L y = b (forward substitution), in place on y (y == b allowed). */
static void solve_lower(int n, const double *L, const double *b, double *y)
{
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
        y[i] = v / L[i * n + i];
    }
}

/* Solve L^T x = y (back substitution). */
static void solve_lower_t(int n, const double *L, const double *y, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
        x[i] = v / L[i * n + i];
    }
}

/* Inverse of an SPD matrix through its Cholesky factor, symmetrised.
 * Returns 0 or -1.  `work` holds n*n doubles.                             */
static int spd_inverse(int n, const double *A, double *Ainv, double *work)
{
    memcpy(work, A, sizeof(double) * (size_t)n * n);
    if (orc_cholesky(n, work)) return -1;
    double *col = (double *)malloc(sizeof(double) * (size_t)n * 2);
    double *e = col + n;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) e[i] = (i == j) ? 1.0 : 0.0;
        solve_lower(n, work, e, col);
        solve_lower_t(n, work, col, col);
        for (int i = 0; i < n; ++i) Ainv[i * n + j] = col[i];
    }
    free(col);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (Ainv[i * n + j] + Ainv[j * n + i]);
            Ainv[i * n + j] = s;
            Ainv[j * n + i] = s;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Row conditional (Algorithm 1, the body of both item loops).              */
/* ------------------------------------------------------------------------ */

/* One conditional draw for a row with d ratings (nbr[e], rc[e]) against the
 * other factor Y (rows x K):  P = Lambda + alpha sum y y^T,
 * b = Lambda mu + alpha sum r' y, L = chol(P), x = L^-T (L^-1 b + z).
 * z (K normals) is supplied by the caller; z = 0 gives the mean P^-1 b.
 * `work` holds K*K + K doubles.  Returns 0, or -1 if P is not SPD.         */
int orc_row_draw_z(int K, double alpha, int64_t d, const int32_t *nbr,
                   const double *rc, const double *Y, const double *mu,
                   const double *Lambda, const double *z, double *x,
                   double *work)
{
    double *P = work;
    double *b = work + (size_t)K * K;
    for (int i = 0; i < K; ++i) {
        double s = 0.0;
        for (int l = 0; l < K; ++l) s += Lambda[i * K + l] * mu[l];
        b[i] = s;
        for (int j = 0; j < K; ++j) P[i * K + j] = Lambda[i * K + j];
    }
    for (int64_t e = 0; e < d; ++e) {
        const double *y = Y + (size_t)nbr[e] * K;
        double r = rc[e];
        for (int i = 0; i < K; ++i) {
            b[i] += alpha * r * y[i];
            for (int j = 0; j <= i; ++j) P[i * K + j] += alpha * y[i] * y[j];
        }
    }
    for (int i = 0; i < K; ++i)
        for (int j = i + 1; j < K; ++j) P[i * K + j] = P[j * K + i];
    if (orc_cholesky(K, P)) return -1;
    solve_lower(K, P, b, x);
    for (int i = 0; i < K; ++i) x[i] += z[i];
    solve_lower_t(K, P, x, x);
    return 0;
}

/* Update the listed rows of X (or all `rows` rows when list == NULL) from
 * their CSR-style neighbour lists ptr/idx/rc against Y, with row noise
 * counter (row, t, stream<<24 | b, 0).  Rows are independent given Y and the
 * hyperparameters, so they run in parallel.  Returns 0 or the negative
 * (1-based) index of the first row whose precision was not SPD.            */
int orc_update_rows(int64_t rows, int K, double alpha, const int64_t *ptr,
                    const int32_t *idx, const double *rc, const double *Y,
                    const double *mu, const double *Lambda, uint64_t seed,
                    uint32_t stream, uint32_t t, const int64_t *list,
                    int64_t n_list, double *X)
{
    int64_t n = list ? n_list : rows;
    int64_t bad = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ((size_t)K * K + 3 * (size_t)K));
        double *z = work + (size_t)K * K + K;
        double *x = z + K;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < n; ++q) {
            int64_t row = list ? list[q] : q;
            int64_t beg = ptr[row], end = ptr[row + 1];
            orc_normals(seed, (uint32_t)row, t, stream, 0u, K, z);
            if (orc_row_draw_z(K, alpha, end - beg, idx + beg, rc + beg, Y, mu,
                               Lambda, z, x, work)) {
#pragma omp critical
                if (!bad || -(row + 1) > bad) bad = -(row + 1);
                continue;
            }
            memcpy(X + (size_t)row * K, x, sizeof(double) * K);
        }
        free(work);
    }
    return bad ? (int)(bad < -2147483647 ? -2147483647 : bad) : 0;
}

/* ------------------------------------------------------------------------ */
/* Normal-Wishart hyperparameter draw (Algorithm 1, "sample hyper-parameters */
/* ... based on V" / "... based on U").                                      */
/* ------------------------------------------------------------------------ */

/* Draw (mu, Lambda) of one side from its n x K factor X.  mu0 (K), W0 (K x K,
 * SPD), beta0 and nu0 are the hyperprior.  The sufficient statistics use two
 * passes over all n rows: xbar, then S = sum (x - xbar)(x - xbar)^T.
 * Returns 0, or -1 if a matrix that must be SPD is not.                     */
int orc_hyper_draw(int64_t n, int K, const double *X, const double *mu0,
                   double beta0, double nu0, const double *W0, uint64_t seed,
                   uint32_t stream, uint32_t t, double *mu, double *Lambda)
{
    size_t KK = (size_t)K * K;
    double *buf = (double *)calloc(8 * KK + 8 * (size_t)K, sizeof(double));
    double *xbar = buf, *S = buf + K, *Winv = S + KK, *Wstar = Winv + KK;
    double *LW = Wstar + KK, *A = LW + KK, *B = A + KK, *work = B + KK;
    double *mustar = work + KK, *zmu = mustar + K, *tmp = zmu + K;
    double *W0inv = tmp + K;
    int rc = -1;

    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < K; ++k) xbar[k] += X[(size_t)i * K + k];
    for (int k = 0; k < K; ++k) xbar[k] /= (double)n;
    for (int64_t i = 0; i < n; ++i) {
        const double *x = X + (size_t)i * K;
        for (int a = 0; a < K; ++a)
            for (int c = 0; c < K; ++c)
                S[a * K + c] += (x[a] - xbar[a]) * (x[c] - xbar[c]);
    }

    double beta_s = beta0 + (double)n;
    double nu_s = nu0 + (double)n;
    for (int k = 0; k < K; ++k)
        mustar[k] = (beta0 * mu0[k] + (double)n * xbar[k]) / beta_s;

    if (spd_inverse(K, W0, W0inv, work)) goto done;
    double shrink = beta0 * (double)n / beta_s;
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < K; ++c)
            Winv[a * K + c] = W0inv[a * K + c] + S[a * K + c] +
                              shrink * (xbar[a] - mu0[a]) * (xbar[c] - mu0[c]);
    if (spd_inverse(K, Winv, Wstar, work)) goto done;

    /* Bartlett: Lambda = (L_W A)(L_W A)^T, A lower triangular with
     * A_kk = sqrt(chi2(nu* - k)), k = 0..K-1, and N(0,1) below the diagonal,
     * taken in row-major order of the strict lower triangle.               */
    memcpy(LW, Wstar, sizeof(double) * KK);
    if (orc_cholesky(K, LW)) goto done;
    for (int k = 0; k < K; ++k)
        A[k * K + k] = sqrt(orc_chi2(seed, stream, t, (uint32_t)k, nu_s - (double)k, NULL));
    {
        int n_low = K * (K - 1) / 2;
        double *zl = (double *)malloc(sizeof(double) * (size_t)(n_low > 0 ? n_low : 1));
        for (int b = 0; 4 * b < n_low; ++b) {
            uint32_t w[4];
            double g[4];
            philox_block(seed, (uint32_t)b, t, (stream << 24) | 1u, 0u, w);
            box_muller4(w, g);
            for (int l = 0; l < 4 && 4 * b + l < n_low; ++l) zl[4 * b + l] = g[l];
        }
        int e = 0;
        for (int r = 1; r < K; ++r)
            for (int c = 0; c < r; ++c) A[r * K + c] = zl[e++];
        free(zl);
    }
    /* B = L_W A (both lower triangular), Lambda = B B^T. */
    for (int r = 0; r < K; ++r)
        for (int c = 0; c <= r; ++c) {
            double s = 0.0;
            for (int m = c; m <= r; ++m) s += LW[r * K + m] * A[m * K + c];
            B[r * K + c] = s;
        }
    for (int r = 0; r < K; ++r)
        for (int c = 0; c <= r; ++c) {
            double s = 0.0;
            for (int m = 0; m <= c; ++m) s += B[r * K + m] * B[c * K + m];
            Lambda[r * K + c] = s;
            Lambda[c * K + r] = s;
        }

    /* mu = mu* + chol(beta* Lambda)^-T z. */
    for (size_t q = 0; q < KK; ++q) work[q] = beta_s * Lambda[q];
    if (orc_cholesky(K, work)) goto done;
    for (int b = 0; 4 * b < K; ++b) {
        uint32_t w[4];
        double g[4];
        philox_block(seed, (uint32_t)b, t, (stream << 24) | 2u, 0u, w);
        box_muller4(w, g);
        for (int l = 0; l < 4 && 4 * b + l < K; ++l) zmu[4 * b + l] = g[l];
    }
    solve_lower_t(K, work, zmu, tmp);
    for (int k = 0; k < K; ++k) mu[k] = mustar[k] + tmp[k];
    rc = 0;
done:
    free(buf);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Initialisation, prediction, centring.                                     */
/* ------------------------------------------------------------------------ */

/* X_ik = scale * z(stream, t = 0, row i, k). */
void orc_init_factor(uint64_t seed, uint32_t stream, int64_t rows, int K,
                     double scale, double *X)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        orc_normals(seed, (uint32_t)i, 0u, stream, 0u, K, X + (size_t)i * K);
        for (int k = 0; k < K; ++k) X[(size_t)i * K + k] *= scale;
    }
}

/* p_e = U_row . V_col + offset for every test pair. */
void orc_predict(int64_t n, int K, const int32_t *row, const int32_t *col,
                 const double *U, const double *V, double offset, double *p)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        const double *u = U + (size_t)row[e] * K;
        const double *v = V + (size_t)col[e] * K;
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += u[k] * v[k];
        p[e] = s + offset;
    }
}

/* Mean of n values, summed sequentially in FP64. */
double orc_mean(int64_t n, const float *v)
{
    double s = 0.0;
    for (int64_t e = 0; e < n; ++e) s += (double)v[e];
    return n ? s / (double)n : 0.0;
}

/* Fold-in of one new user (not a step of Algorithm 1: the serving
 * extension): for each of S stored samples s, draw u_s from the row
 * conditional against V^(s) with prior (mu^(s), Lambda^(s)) and noise
 * counter (lo32(req), s, stream<<24 | b, hi32(req)); score every movie with
 * p_sj = u_s . v_j^(s) + offset; return per-movie mean over s and variance
 * 1/alpha + (1/S) sum_s (p_sj - mean_j)^2.  U_out (S x K) receives the
 * draws.  Returns 0 or -1.                                                  */
int orc_foldin(int S, int64_t N, int K, double alpha, int64_t d,
               const int32_t *movie, const double *rc, const double *Vs,
               const double *mus, const double *Lambdas, uint64_t seed,
               uint32_t stream, uint64_t req, double offset, double *U_out,
               double *mean, double *var)
{
    double *work = (double *)malloc(sizeof(double) * ((size_t)K * K + 2 * (size_t)K));
    double *z = work + (size_t)K * K + K;
    double *P = (double *)malloc(sizeof(double) * (size_t)S * N);
    int rc_out = 0;
    for (int s = 0; s < S; ++s) {
        const double *V = Vs + (size_t)s * N * K;
        orc_normals(seed, (uint32_t)req, (uint32_t)s, stream, (uint32_t)(req >> 32), K, z);
        if (orc_row_draw_z(K, alpha, d, movie, rc, V, mus + (size_t)s * K,
                           Lambdas + (size_t)s * K * K, z, U_out + (size_t)s * K, work)) {
            rc_out = -1;
            goto out;
        }
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += U_out[(size_t)s * K + k] * V[(size_t)j * K + k];
            P[(size_t)s * N + j] = acc + offset;
        }
    }
    for (int64_t j = 0; j < N; ++j) {
        double m = 0.0;
        for (int s = 0; s < S; ++s) m += P[(size_t)s * N + j];
        m /= (double)S;
        double v = 0.0;
        for (int s = 0; s < S; ++s) {
            double q = P[(size_t)s * N + j] - m;
            v += q * q;
        }
        mean[j] = m;
        var[j] = 1.0 / alpha + v / (double)S;
    }
out:
    free(P);
    free(work);
    return rc_out;
}

#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int n) { omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int n) { (void)n; }
int orc_max_threads(void) { return 1; }
#endif
