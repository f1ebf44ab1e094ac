/*
 * CPU oracle for the Kolmogorov-Smirnov change-point detection of MT4G
 * (arXiv 2511.05958, Section "Benchmarks and Autoevaluation", size benchmarks,
 * workflow step 4 "The K-S test"; Section "Background", K-S test and eq. 1).
 *
 * TEST INFRASTRUCTURE. This library is a slow, plain, obviously-correct
 * restatement of the method, used only to check the GPU path: only tests/,
 * __graft_entry__.smoke() and bench.py's cpu_baseline leg may load or call it.
 * It shares no code, header, table or helper with the HIP path.
 *
 * What one series is: the 2-D timing array of one size sweep, K array sizes
 * (rows) x the first N load latencies of each size (columns), uint32 cycles,
 * row-major.
 *
 * Method, in the paper's order:
 *  1. Eq. 2 geometric-mapping reduction: S_i = sqrt(sum_j (r_ij - min r)^2)
 *     with min r the minimum over the whole 2-D array and j running over the
 *     N stored latencies. The oracle keeps Q_i = S_i^2 as an exact 128-bit
 *     integer: sqrt is strictly increasing and the K-S statistic depends on
 *     ranks only, so the statistic is the same and exact.
 *  2. Every index c = 1..K-1 of S is a candidate change point. The K-S two
 *     sample test compares the values below the candidate (rows [0, c), n = c
 *     values) with the values from the candidate on (rows [c, K), m = K - c
 *     values): D_c = max_x |F(x) - G(x)| with the empirical distribution
 *     functions F, G. The oracle keeps the numerator U_c = n m D_c, an
 *     integer.
 *  3. The change point is the candidate of highest significance, i.e. the
 *     largest lambda_c = D_c sqrt(n m / (n + m)) (equivalently the smallest
 *     asymptotic p-value); ties go to the smallest c.
 *  4. Eq. 1 critical value d_alpha = sqrt(-1/2 ln(alpha/2) (n+m)/(n m))
 *     (the printed formula lacks the minus sign; this is the one-term
 *     inverse of the Kolmogorov tail). H0 is denied iff D > d_alpha, which
 *     is U^2 > c_alpha n m K with c_alpha = -1/2 ln(alpha/2).
 *  5. The significance reported as confidence: the asymptotic Kolmogorov
 *     p-value Q_KS(lambda) of the winner.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Result of one series (the oracle's own layout, 48 bytes). */
typedef struct oracle_result {
  uint32_t cp;     /* first row of the higher side, c* */
  uint32_t n, m;   /* sizes of the lower and higher side */
  uint32_t U;      /* D numerator: U = n m D */
  double D;        /* U / (n m) */
  double lambda;   /* sqrt(U^2 / (n m K)) */
  double p;        /* asymptotic Kolmogorov p-value of lambda */
  uint32_t significant;
  uint32_t status; /* 0 ok, 1 bad shape (K < 2 or N < 1) */
} oracle_result;

/* ---- step 1: eq. 2, exact ---- */

/* Global minimum of the 2-D array and Q_i = sum_j (r_ij - min)^2 for every
 * row, as (lo, hi) 64-bit halves of a 128-bit integer. */
void oracle_reduce(const uint32_t *r, uint32_t K, uint32_t N, uint32_t *gmin, uint64_t *Q_lo,
                   uint64_t *Q_hi) {
  uint32_t mn = 0xffffffffu;
  for (uint64_t t = 0; t < (uint64_t)K * N; ++t)
    if (r[t] < mn) mn = r[t];
  for (uint32_t i = 0; i < K; ++i) {
    u128 q = 0;
    for (uint32_t j = 0; j < N; ++j) {
      uint64_t d = (uint64_t)r[(uint64_t)i * N + j] - mn;
      q += (u128)(d * d);
    }
    Q_lo[i] = (uint64_t)q;
    Q_hi[i] = (uint64_t)(q >> 64);
  }
  *gmin = mn;
}

/* ---- step 2: two-sample K-S numerator of one split ---- */

static int cmp_u128(const void *a, const void *b) {
  u128 x = *(const u128 *)a, y = *(const u128 *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* U_c = max over all real x of |i(x) m - j(x) n|, where i(x) counts lower-side
 * values <= x and j(x) higher-side values <= x. Both sides are sorted and
 * walked together; the difference is taken after every complete group of
 * equal values, which is where the empirical distribution functions step. */
static uint64_t split_U(const u128 *Q, uint32_t K, uint32_t c, u128 *A, u128 *B) {
  const uint32_t n = c, m = K - c;
  memcpy(A, Q, sizeof(u128) * n);
  memcpy(B, Q + c, sizeof(u128) * m);
  qsort(A, n, sizeof(u128), cmp_u128);
  qsort(B, m, sizeof(u128), cmp_u128);
  uint32_t i = 0, j = 0;
  uint64_t U = 0;
  while (i < n || j < m) {
    u128 x;
    if (i < n && (j >= m || A[i] <= B[j]))
      x = A[i];
    else
      x = B[j];
    while (i < n && A[i] == x) ++i;
    while (j < m && B[j] == x) ++j;
    int64_t d = (int64_t)i * m - (int64_t)j * n;
    uint64_t ad = (uint64_t)(d < 0 ? -d : d);
    if (ad > U) U = ad;
  }
  return U;
}

uint64_t oracle_split_U(const uint64_t *Q_lo, const uint64_t *Q_hi, uint32_t K, uint32_t c) {
  if (K < 2 || c < 1 || c >= K) return 0;
  u128 *Q = malloc(sizeof(u128) * K * 3);
  for (uint32_t i = 0; i < K; ++i) Q[i] = ((u128)Q_hi[i] << 64) | Q_lo[i];
  uint64_t U = split_U(Q, K, c, Q + K, Q + 2 * K);
  free(Q);
  return U;
}

/* ---- step 4: eq. 1 constant ---- */

double oracle_c_alpha(double alpha) { return -0.5 * log(alpha / 2.0); }

/* ---- step 5: asymptotic Kolmogorov p-value ---- */

/* Q_KS(lambda) = 2 sum_{k>=1} (-1)^(k-1) exp(-2 k^2 lambda^2)
 *             = 1 - sqrt(2 pi)/lambda sum_{k>=1} exp(-(2k-1)^2 pi^2 / (8 lambda^2)),
 * the first form for lambda >= 1, the second below; each series stops once a
 * term falls under 1e-20 of the running sum. Flushed to 0 when
 * 2 lambda^2 > 700 (the first term is then below 1e-304). Evaluated in long
 * double from the double lambda^2. */
double oracle_kolmogorov(double lambda2) {
  if (!(lambda2 > 0.0)) return 1.0;
  if (2.0 * lambda2 > 700.0) return 0.0;
  const long double l2 = (long double)lambda2;
  const long double lam = sqrtl(l2);
  long double sum = 0.0L;
  if (lam >= 1.0L) {
    for (int k = 1; k <= 200; ++k) {
      long double term = expl(-2.0L * (long double)k * (long double)k * l2);
      sum += (k & 1) ? term : -term;
      if (term < 1e-20L * fabsl(sum)) break;
    }
    return (double)(2.0L * sum);
  } else {
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 1; k <= 200; ++k) {
      long double o = (long double)(2 * k - 1);
      long double term = expl(-o * o * pi * pi / (8.0L * l2));
      sum += term;
      if (term < 1e-20L * sum) break;
    }
    return (double)(1.0L - sqrtl(2.0L * pi) / lam * sum);
  }
}

/* ---- one series ---- */

int oracle_scan_series(const uint32_t *r, uint32_t K, uint32_t N, double alpha, oracle_result *res,
                       uint32_t *allU /* K entries or NULL; allU[c] = U_c, allU[0] = 0 */) {
  memset(res, 0, sizeof(*res));
  if (K < 2 || N < 1) {
    res->status = 1;
    return 1;
  }
  uint64_t *ql = malloc(sizeof(uint64_t) * K * 2);
  u128 *Q = malloc(sizeof(u128) * K * 3);
  uint64_t *U = malloc(sizeof(uint64_t) * K);
  uint32_t mn;
  oracle_reduce(r, K, N, &mn, ql, ql + K);
  for (uint32_t i = 0; i < K; ++i) Q[i] = ((u128)ql[K + i] << 64) | ql[i];

  U[0] = 0;
  for (uint32_t c = 1; c < K; ++c) U[c] = split_U(Q, K, c, Q + K, Q + 2 * K);

  /* step 3: argmax of U_c^2 / (c (K - c)), compared exactly by cross-multiplying */
  uint32_t best = 1;
  for (uint32_t c = 2; c < K; ++c) {
    u128 lhs = (u128)U[c] * U[c] * ((u128)best * (K - best));
    u128 rhs = (u128)U[best] * U[best] * ((u128)c * (K - c));
    if (lhs > rhs) best = c;
  }
  const uint32_t n = best, m = K - best;
  const uint64_t Ub = U[best];
  const double U2 = (double)(Ub * Ub);
  const double nmK = (double)((uint64_t)n * m * K);
  res->cp = best;
  res->n = n;
  res->m = m;
  res->U = (uint32_t)Ub;
  res->D = (double)Ub / (double)((uint64_t)n * m);
  const double lambda2 = U2 / nmK;
  res->lambda = sqrt(lambda2);
  res->p = Ub == 0 ? 1.0 : oracle_kolmogorov(lambda2);
  res->significant = U2 > oracle_c_alpha(alpha) * nmK;
  if (allU)
    for (uint32_t c = 0; c < K; ++c) allU[c] = (uint32_t)U[c];
  free(ql);
  free(Q);
  free(U);
  return 0;
}

/* ---- a batch over a thread pool ---- */

typedef struct {
  const uint32_t *samples;
  const uint64_t *offsets;
  const uint32_t *Ks, *Ns;
  uint32_t num;
  double alpha;
  oracle_result *res;
  uint32_t *allU;
  const uint64_t *allU_off;
  uint32_t next;
  pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *job = arg;
  for (;;) {
    pthread_mutex_lock(&job->mu);
    uint32_t s = job->next++;
    pthread_mutex_unlock(&job->mu);
    if (s >= job->num) break;
    oracle_scan_series(job->samples + job->offsets[s], job->Ks[s], job->Ns[s], job->alpha, &job->res[s],
                       job->allU ? job->allU + job->allU_off[s] : NULL);
  }
  return NULL;
}

int oracle_scan_batch(const uint32_t *samples, const uint64_t *offsets, const uint32_t *Ks,
                      const uint32_t *Ns, uint32_t num, double alpha, oracle_result *res, uint32_t *allU,
                      const uint64_t *allU_off, int threads) {
  batch_job job = {samples, offsets, Ks, Ns, num, alpha, res, allU, allU_off, 0};
  pthread_mutex_init(&job.mu, NULL);
  if (threads < 1) threads = 1;
  pthread_t *th = malloc(sizeof(pthread_t) * threads);
  for (int t = 1; t < threads; ++t) pthread_create(&th[t], NULL, batch_worker, &job);
  batch_worker(&job);
  for (int t = 1; t < threads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&job.mu);
  return 0;
}

unsigned oracle_result_size(void) { return (unsigned)sizeof(oracle_result); }

/* ---- learned-proposal inputs (project-defined; the paper has no learned stage) ----
 *
 * Per-row quantile features: for each row i, the row's N samples sorted
 * ascending, the order statistics x_(floor(k (N-1) / 10)) for k = 1..9 (the
 * nine deciles), each mapped to f = (float)((double)(x - m) / max(m, 1)) with
 * m the minimum of the whole 2-D array (the eq. 2 global minimum). */

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

void oracle_features(const uint32_t *r, uint32_t K, uint32_t N, float *out /* K*9 */) {
  uint32_t mn = 0xffffffffu;
  for (uint64_t t = 0; t < (uint64_t)K * N; ++t)
    if (r[t] < mn) mn = r[t];
  const double denom = (double)(mn > 1 ? mn : 1);
  uint32_t *row = malloc(sizeof(uint32_t) * (N ? N : 1));
  for (uint32_t i = 0; i < K; ++i) {
    memcpy(row, r + (uint64_t)i * N, sizeof(uint32_t) * N);
    qsort(row, N, sizeof(uint32_t), cmp_u32);
    for (uint32_t k = 1; k <= 9; ++k) {
      uint32_t x = row[(uint64_t)k * (N - 1) / 10];
      out[(uint64_t)i * 9 + (k - 1)] = (float)((double)(x - mn) / denom);
    }
  }
  free(row);
}
