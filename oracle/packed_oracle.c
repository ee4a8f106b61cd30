/*
 * CPU oracle for the packed symmetric tensor of tensor-kernel regression.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded FP64 C written
 * directly from the definitions; it shares no code with the GPU library and
 * may be called only by the tests, the smoke check and the benchmark's CPU
 * baseline leg.
 *
 * Storage (Section 5, the nested-loop listing and eq. b_tensor4): an order-m
 * symmetric tensor over n points keeps one value per sorted index tuple
 * t_0 <= t_1 <= ... <= t_{m-1} < n, in the order of m nested loops where each
 * loop starts at the previous loop's index and the last index runs fastest.
 * There are C(n+m-1, m) such tuples.
 *
 * Every routine walks the tuples in that order with next_tuple(), so the
 * position of a tuple in the flat array is simply its visit count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_ORDER 16

/* Successor of a sorted tuple in nested-loop order; 0 once past the last. */
static int next_tuple(int64_t *t, int m, int64_t n)
{
    int p = m - 1;
    while (p >= 0 && t[p] == n - 1)
        p--;
    if (p < 0)
        return 0;
    t[p]++;
    for (int q = p + 1; q < m; q++)
        t[q] = t[p];
    return 1;
}

static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++)
        f *= (double)i;
    return f;
}

/* prod over distinct values v of (multiplicity of v in t)! ; t is sorted. */
static double multiplicity_factorials(const int64_t *t, int m)
{
    double prod = 1.0;
    int run = 1;
    for (int p = 1; p <= m; p++) {
        if (p < m && t[p] == t[p - 1]) {
            run++;
        } else {
            prod *= factorial(run);
            run = 1;
        }
    }
    return prod;
}

/*
 * Number of ordered index tuples (i_1..i_m) whose sorted form is t:
 * m! / prod_v c_v!.
 */
double or_orderings(const int64_t *t, int m)
{
    return factorial(m) / multiplicity_factorials(t, m);
}

/*
 * Build the packed tensor of a tensor kernel (Section 4):
 *   linear:       k(x_1..x_m) = sum_j x_{1j} ... x_{mj}
 *   polynomial:   (linear)^s                       (eq. poly_tensor), s = kparam
 *   exponential:  exp(linear)
 * X is row-major [n x d].  K receives C(n+m-1, m) values.
 */
int or_build_packed(const double *X, int64_t n, int64_t d, int m, int kernel,
                    double kparam, double *K)
{
    if (m < 1 || m > OR_MAX_ORDER || n < 1 || d < 1)
        return -1;
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    do {
        double s = 0.0;
        for (int64_t j = 0; j < d; j++) {
            double prod = 1.0;
            for (int p = 0; p < m; p++)
                prod *= X[t[p] * d + j];
            s += prod;
        }
        if (kernel == 1) {
            double r = 1.0;
            for (int k = 0; k < (int)kparam; k++)
                r *= s;
            s = r;
        } else if (kernel == 2) {
            s = exp(s);
        }
        K[e++] = s;
    } while (next_tuple(t, m, n));
    return 0;
}

/*
 * Contraction g = K . alpha^{m-1}:  g_a = sum_{i_2..i_m} K_{a i_2..i_m} alpha_{i_2}..alpha_{i_m}
 * (the gradient of the first term of eq. dual_tensor_kernel).
 *
 * Every ordered tuple (a, i_2..i_m) has a sorted form t and appears once per
 * distinct ordering.  Fixing the position p of a in t, the orderings that put
 * t_p first number (m-1)!/prod_v c_v! (counting each equal value's slots
 * separately), so each sorted tuple adds
 *     w(t) * K_t * prod_{q != p} alpha_{t_q},   w(t) = (m-1)!/prod_v c_v!,
 * to g_{t_p} for every position p = 0..m-1.
 */
int or_contract_packed(const double *K, int64_t n, int m, const double *alpha, double *g)
{
    if (m < 1 || m > OR_MAX_ORDER || n < 1)
        return -1;
    for (int64_t i = 0; i < n; i++)
        g[i] = 0.0;
    const double fm1 = factorial(m - 1);
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    do {
        const double w = fm1 / multiplicity_factorials(t, m);
        const double kv = K[e++];
        for (int p = 0; p < m; p++) {
            double prod = 1.0;
            for (int q = 0; q < m; q++)
                if (q != p)
                    prod *= alpha[t[q]];
            g[t[p]] += w * kv * prod;
        }
    } while (next_tuple(t, m, n));
    return 0;
}

/*
 * Directional derivative of the contraction: h = d/de g(alpha + e v) at e = 0,
 * i.e. h = (m-1) K x_2 v x_3 alpha ... x_m alpha.  Differentiating each
 * product term of or_contract_packed gives, per sorted tuple and position p,
 *     w(t) K_t sum_{q != p} v_{t_q} prod_{r != p, q} alpha_{t_r}   added to h_{t_p}.
 */
int or_hvp_packed(const double *K, int64_t n, int m, const double *alpha,
                  const double *v, double *h)
{
    if (m < 1 || m > OR_MAX_ORDER || n < 1)
        return -1;
    for (int64_t i = 0; i < n; i++)
        h[i] = 0.0;
    const double fm1 = factorial(m - 1);
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    do {
        const double w = fm1 / multiplicity_factorials(t, m);
        const double kv = K[e++];
        for (int p = 0; p < m; p++) {
            double acc = 0.0;
            for (int q = 0; q < m; q++) {
                if (q == p)
                    continue;
                double prod = v[t[q]];
                for (int r = 0; r < m; r++)
                    if (r != p && r != q)
                        prod *= alpha[t[r]];
                acc += prod;
            }
            h[t[p]] += w * kv * acc;
        }
    } while (next_tuple(t, m, n));
    return 0;
}

/*
 * Jacobian of the contraction (n x n, row-major): H_{ab} = d g_a / d alpha_b
 * = (m-1) sum K_{a b i_3..i_m} alpha_{i_3}..alpha_{i_m}.  Per sorted tuple,
 * position p and another position q, adds w(t) K_t prod_{r != p,q} alpha_{t_r}
 * to H[t_p][t_q].
 */
int or_jacobian_packed(const double *K, int64_t n, int m, const double *alpha, double *H)
{
    if (m < 2 || m > OR_MAX_ORDER || n < 1)
        return -1;
    for (int64_t i = 0; i < n * n; i++)
        H[i] = 0.0;
    const double fm1 = factorial(m - 1);
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    do {
        const double w = fm1 / multiplicity_factorials(t, m);
        const double kv = K[e++];
        for (int p = 0; p < m; p++) {
            for (int q = 0; q < m; q++) {
                if (q == p)
                    continue;
                double prod = 1.0;
                for (int r = 0; r < m; r++)
                    if (r != p && r != q)
                        prod *= alpha[t[r]];
                H[t[p] * n + t[q]] += w * kv * prod;
            }
        }
    } while (next_tuple(t, m, n));
    return 0;
}

/*
 * Full-tensor multilinear form <K, alpha^{(x)m}> = sum_{i_1..i_m} K_{i_1..i_m} alpha_{i_1}..alpha_{i_m}:
 * each sorted tuple stands for m!/prod_v c_v! ordered tuples.
 */
double or_multilinear_packed(const double *K, int64_t n, int m, const double *alpha)
{
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    double s = 0.0;
    do {
        double prod = 1.0;
        for (int p = 0; p < m; p++)
            prod *= alpha[t[p]];
        s += or_orderings(t, m) * K[e++] * prod;
    } while (next_tuple(t, m, n));
    return s;
}

/* Write every sorted tuple, in storage order, into T[count x m] (small n only). */
int64_t or_enumerate(int64_t n, int m, int64_t *T, int64_t cap)
{
    int64_t t[OR_MAX_ORDER];
    for (int p = 0; p < m; p++)
        t[p] = 0;
    int64_t e = 0;
    do {
        if (e >= cap)
            return -1;
        for (int p = 0; p < m; p++)
            T[e * m + p] = t[p];
        e++;
    } while (next_tuple(t, m, n));
    return e;
}

/* Value of one packed entry, computed alone (used to check sampled entries). */
double or_kernel_entry(const double *X, int64_t d, const int64_t *t, int m, int kernel,
                       double kparam)
{
    double s = 0.0;
    for (int64_t j = 0; j < d; j++) {
        double prod = 1.0;
        for (int p = 0; p < m; p++)
            prod *= X[t[p] * d + j];
        s += prod;
    }
    if (kernel == 1) {
        double r = 1.0;
        for (int k = 0; k < (int)kparam; k++)
            r *= s;
        s = r;
    } else if (kernel == 2) {
        s = exp(s);
    }
    return s;
}
