/*
 * Test infrastructure only (the oracle).  Nothing in the product library
 * links or calls this file; only tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.
 *
 * Plain FP64 state-vector simulation of an open-chain brickwork circuit.
 * It computes psi(x) = <x| U |0^n> with
 *     U = L_d E_d L_{d-1} ... E_1 L_0
 * directly from that definition (problem statement of Sec. 2.2, the
 * amplitude equation; circuit family of Sec. 2.1): every one-qubit layer
 * L_l is n strided 2x2 updates, every entangler of layer E_l is applied to
 * its qubit pair (CZ as a sign flip on |11>, a dense 4x4 otherwise).
 * No blocking, no fusion, no reordering.
 *
 * Conventions: qubit j is bit (n-1-j) of the state index, so a bitstring
 * x_0 x_1 ... x_{n-1} read MSB-first is its index.  Complex numbers are
 * interleaved (re, im) doubles.  one_qubit[((l*n + q)*4 + 2*r + c)] is
 * entry [r][c] (row = out, column = in) of L_l on qubit q.  A dense 4x4
 * acts on basis index 2*x_q + x_{q+1}.  A gate with q = n-1 acts on the
 * ring's wrap pair (n-1, 0) (periodic geometry of Sec. 6.3), basis index
 * 2*x_{n-1} + x_0.
 *
 * `mutation` plants a deliberate mistake; it exists so that the oracle's
 * own tests can show that their pins catch such mistakes.  0 = none.
 *   1: skip the final one-qubit layer L_d
 *   2: apply every one-qubit gate transposed
 *   3: CZ flips the sign of |01> instead of |11>
 *   4: apply entangling layer l+1 before one-qubit layer l
 *   5: map qubit j to bit j (reversed qubit order)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) {
    cplx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static inline cplx cadd(cplx a, cplx b) {
    cplx r = { a.re + b.re, a.im + b.im };
    return r;
}

static int bit_of(int n, int q, int mutation) {
    return mutation == 5 ? q : n - 1 - q;
}

static void apply_1q(cplx *psi, int n, int q, const cplx m_in[4], int mutation) {
    cplx m[4] = { m_in[0], m_in[1], m_in[2], m_in[3] };
    if (mutation == 2) { m[1] = m_in[2]; m[2] = m_in[1]; }
    const int64_t stride = (int64_t)1 << bit_of(n, q, mutation);
    const int64_t half = (int64_t)1 << (n - 1);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < half; ++p) {
        /* index with a 0 inserted at the target bit */
        int64_t lo = p & (stride - 1);
        int64_t i0 = ((p - lo) << 1) | lo;
        int64_t i1 = i0 | stride;
        cplx a0 = psi[i0], a1 = psi[i1];
        psi[i0] = cadd(cmul(m[0], a0), cmul(m[1], a1));
        psi[i1] = cadd(cmul(m[2], a0), cmul(m[3], a1));
    }
}

/* The pair of a gate with upper qubit q is (q, q+1); q = n-1 is the ring's
 * wrap pair (n-1, 0). */
static int partner(int n, int q) { return q + 1 < n ? q + 1 : 0; }

static void apply_cz(cplx *psi, int n, int q, int mutation) {
    const int64_t s1 = (int64_t)1 << bit_of(n, q, mutation);               /* qubit q   */
    const int64_t s2 = (int64_t)1 << bit_of(n, partner(n, q), mutation);   /* its partner */
    const int64_t dim = (int64_t)1 << n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        int hit = mutation == 3 ? (!(i & s1) && (i & s2)) : ((i & s1) && (i & s2));
        if (hit) { psi[i].re = -psi[i].re; psi[i].im = -psi[i].im; }
    }
}

static void apply_dense4(cplx *psi, int n, int q, const cplx m[16], int mutation) {
    const int64_t s1 = (int64_t)1 << bit_of(n, q, mutation);
    const int64_t s2 = (int64_t)1 << bit_of(n, partner(n, q), mutation);
    const int64_t dim = (int64_t)1 << n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if ((i & s1) || (i & s2)) continue;
        int64_t idx[4] = { i, i | s2, i | s1, i | s1 | s2 };  /* 2*x_q + x_{q+1} */
        cplx a[4], r[4];
        for (int u = 0; u < 4; ++u) a[u] = psi[idx[u]];
        for (int o = 0; o < 4; ++o) {
            cplx acc = { 0.0, 0.0 };
            for (int u = 0; u < 4; ++u) acc = cadd(acc, cmul(m[4 * o + u], a[u]));
            r[o] = acc;
        }
        for (int u = 0; u < 4; ++u) psi[idx[u]] = r[u];
    }
}

static void apply_layer(cplx *psi, int n, int layer, int n_g, const int32_t *g_layer,
                        const int32_t *g_q, const int32_t *g_kind, const cplx *g_mat,
                        int mutation) {
    for (int g = 0; g < n_g; ++g) {
        if (g_layer[g] != layer) continue;
        if (g_kind[g] == 0) apply_cz(psi, n, g_q[g], mutation);
        else apply_dense4(psi, n, g_q[g], g_mat + 16 * (int64_t)g, mutation);
    }
}

/* Full state vector.  psi must hold 2^n complex numbers.  Returns 0 on
 * success, -1 on bad arguments. */
int oracle_statevector(int n, int d, const double *one_qubit, int n_g,
                       const int32_t *g_layer, const int32_t *g_q, const int32_t *g_kind,
                       const double *g_mat, int mutation, double *psi_out) {
    if (n < 1 || n > 34 || d < 0) return -1;
    for (int g = 0; g < n_g; ++g)
        if (g_layer[g] < 1 || g_layer[g] > d || g_q[g] < 0 || g_q[g] >= n || (g_q[g] == n - 1 && n < 3))
            return -1;
    cplx *psi = (cplx *)psi_out;
    const cplx *L = (const cplx *)one_qubit;
    const cplx *M = (const cplx *)g_mat;
    const int64_t dim = (int64_t)1 << n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) { psi[i].re = 0.0; psi[i].im = 0.0; }
    psi[0].re = 1.0;
    for (int l = 0; l <= d; ++l) {
        if (mutation == 4 && l < d)
            apply_layer(psi, n, l + 1, n_g, g_layer, g_q, g_kind, M, mutation);
        if (!(mutation == 1 && l == d))
            for (int q = 0; q < n; ++q)
                apply_1q(psi, n, q, L + ((int64_t)l * n + q) * 4, mutation);
        if (mutation != 4 && l < d)
            apply_layer(psi, n, l + 1, n_g, g_layer, g_q, g_kind, M, mutation);
    }
    return 0;
}
