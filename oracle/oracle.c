/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct complex128 state-vector simulator on the
 * host.  It is the reference the GPU library is checked against; nothing in
 * the product path may link, load or call it (only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark do).  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Conventions (qHiPSTER, Sec. 2 "Background"):
 *   - the state of n qubits is 2^n complex doubles stored in index order;
 *   - qubit q is bit q of the amplitude index, so a gate on qubit k pairs
 *     amplitudes whose indices differ in bit k, a stride of 2^k apart;
 *   - a 2x2 gate Q is passed as 8 doubles, row-major (q11, q12, q21, q22),
 *     each as (re, im), and acts on the column (alpha_{..0_k..}, alpha_{..1_k..})
 *     as in Eq. (2);
 *   - the controlled gate of Eq. (3) applies Q to the target only where the
 *     control bit is 1.
 *
 * Arithmetic is IEEE double with C99 complex numbers; the build uses
 * -fcx-limited-range (textbook complex product) and -ffp-contract=off.
 * Reductions accumulate in long double (x87 80-bit) in index order.
 *
 * OpenMP may split the independent iterations of a loop over threads.
 * Every amplitude is still computed by exactly the formula below, so the
 * thread count never changes a result.
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

static int g_threads = 1;

/* Number of OpenMP threads used by the loops below (1 = serial). */
void oracle_set_threads(int t) { g_threads = t < 1 ? 1 : t; }

int oracle_get_threads(void) { return g_threads; }

static cplx entry(const double* q, int r, int c) {
  return q[4 * r + 2 * c] + I * q[4 * r + 2 * c + 1];
}

/* |0...0> (or any computational basis state |idx>). */
void oracle_init_basis(cplx* a, int n, uint64_t idx) {
  const uint64_t N = 1ull << n;
  for (uint64_t i = 0; i < N; i++) a[i] = 0.0;
  a[idx] = 1.0;
}

/*
 * Index of the p-th pair's first member for target k: p with a 0 bit
 * inserted at position k.  Its partner differs only in bit k.
 */
static int64_t pair_low(int64_t p, int k) {
  const int64_t below = p & (((int64_t)1 << k) - 1);
  return ((p - below) << 1) | below;
}

/*
 * Single-qubit gate on qubit k, Eq. (2): every index pair (i0, i1) that
 * differs only in bit k, with bit k of i0 equal to 0, takes the 2x2 matrix
 * product (a[i0], a[i1]) <- Q (a[i0], a[i1]).  There are 2^(n-1) such pairs
 * and each is updated independently of the others.
 */
void oracle_apply_1q(cplx* a, int n, int k, const double* q) {
  const cplx q11 = entry(q, 0, 0), q12 = entry(q, 0, 1);
  const cplx q21 = entry(q, 1, 0), q22 = entry(q, 1, 1);
  const int64_t npairs = (int64_t)1 << (n - 1), bit = (int64_t)1 << k;
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
  for (int64_t p = 0; p < npairs; p++) {
    const int64_t i0 = pair_low(p, k), i1 = i0 | bit;
    const cplx x = a[i0], y = a[i1];
    a[i0] = q11 * x + q12 * y;
    a[i1] = q21 * x + q22 * y;
  }
}

/*
 * Controlled-Q with control c and target t, Eq. (3): the pairs of Eq. (2)
 * for target t, of which only those whose control bit is 1 are updated;
 * the others keep their amplitudes.
 */
void oracle_apply_cu(cplx* a, int n, int c, int t, const double* q) {
  const cplx q11 = entry(q, 0, 0), q12 = entry(q, 0, 1);
  const cplx q21 = entry(q, 1, 0), q22 = entry(q, 1, 1);
  const int64_t npairs = (int64_t)1 << (n - 1), bit = (int64_t)1 << t;
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
  for (int64_t p = 0; p < npairs; p++) {
    const int64_t i0 = pair_low(p, t), i1 = i0 | bit;
    if (((i0 >> c) & 1) == 0) continue;
    const cplx x = a[i0], y = a[i1];
    a[i0] = q11 * x + q12 * y;
    a[i1] = q21 * x + q22 * y;
  }
}

/*
 * A gate on a block of k qubits: u is the 2^k x 2^k matrix, row-major, each
 * entry (re, im); targets[j] is the qubit that bit j of u's row and column
 * index refers to.  The same reading of Eq. (2) for k qubits: every group
 * of 2^k amplitudes whose indices differ only in the target bits, listed in
 * the order of that k-bit index, is replaced by u times the group.
 */
void oracle_apply_kq(cplx* a, int n, int k, const int* targets, const double* u) {
  const int64_t N = (int64_t)1 << n, K = (int64_t)1 << k;
  int64_t tmask = 0;
  for (int j = 0; j < k; j++) tmask |= (int64_t)1 << targets[j];
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
  for (int64_t i = 0; i < N; i++) {
    if (i & tmask) continue; /* i is the group's member with every target bit 0 */
    int64_t idx[32];
    cplx v[32];
    for (int64_t r = 0; r < K; r++) {
      int64_t x = i;
      for (int j = 0; j < k; j++)
        if ((r >> j) & 1) x |= (int64_t)1 << targets[j];
      idx[r] = x;
      v[r] = a[x];
    }
    for (int64_t r = 0; r < K; r++) {
      cplx s = 0;
      for (int64_t c = 0; c < K; c++) s += (u[2 * (r * K + c)] + I * u[2 * (r * K + c) + 1]) * v[c];
      a[idx[r]] = s;
    }
  }
}

/*
 * Qubit reordering (the state reordering of Sec. 6): qubit q is relabelled
 * perm[q], so the amplitude at index i moves to the index j that has bit
 * perm[q] equal to bit q of i, for every q.  perm must be a permutation of
 * 0 .. n-1.  Out of place through a temporary copy of the state.
 * Returns 0, or -1 if the copy cannot be allocated.
 */
int oracle_permute_qubits(cplx* a, int n, const int* perm) {
  const int64_t N = (int64_t)1 << n;
  cplx* src = (cplx*)malloc((size_t)N * sizeof(cplx));
  if (!src) return -1;
  memcpy(src, a, (size_t)N * sizeof(cplx));
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
  for (int64_t i = 0; i < N; i++) {
    int64_t j = 0;
    for (int q = 0; q < n; q++)
      if ((i >> q) & 1) j |= (int64_t)1 << perm[q];
    a[j] = src[i];
  }
  free(src);
  return 0;
}

/*
 * Measurement probabilities: full[i] = |a_i|^2 (if full != NULL),
 * p1[k] = sum of |a_i|^2 over indices with bit k set (the probability of
 * reading qubit k as 1), and *norm2 = sum of all |a_i|^2.
 */
void oracle_probabilities(const cplx* a, int n, double* p1, double* norm2,
                          double* full) {
  const uint64_t N = 1ull << n;
  long double acc[64];
  long double tot = 0.0L;
  for (int k = 0; k < n; k++) acc[k] = 0.0L;
  for (uint64_t i = 0; i < N; i++) {
    const double re = creal(a[i]), im = cimag(a[i]);
    const double p = re * re + im * im;
    if (full) full[i] = p;
    tot += p;
    for (int k = 0; k < n; k++)
      if ((i >> k) & 1) acc[k] += p;
  }
  for (int k = 0; k < n; k++) p1[k] = (double)acc[k];
  if (norm2) *norm2 = (double)tot;
}

/* <a|b> = sum_i conj(a_i) b_i, accumulated in long double, index order. */
void oracle_inner(const cplx* a, const cplx* b, int n, double* re, double* im) {
  const uint64_t N = 1ull << n;
  long double sr = 0.0L, si = 0.0L;
  for (uint64_t i = 0; i < N; i++) {
    const double ar = creal(a[i]), ai = cimag(a[i]);
    const double br = creal(b[i]), bi = cimag(b[i]);
    sr += (long double)ar * br + (long double)ai * bi;
    si += (long double)ar * bi - (long double)ai * br;
  }
  *re = (double)sr;
  *im = (double)si;
}

/*
 * Pauli matrices as 2x2 gates in the layout above; code 1 = X, 2 = Y, 3 = Z.
 * The identity (code 0) is never applied.
 */
static void pauli_matrix(int code, double* q) {
  memset(q, 0, 8 * sizeof(double));
  if (code == 1) {        /* X = [[0, 1], [1, 0]] */
    q[2] = 1.0;
    q[4] = 1.0;
  } else if (code == 2) { /* Y = [[0, -i], [i, 0]] */
    q[3] = -1.0;
    q[5] = 1.0;
  } else {                /* Z = [[1, 0], [0, -1]] */
    q[0] = 1.0;
    q[6] = -1.0;
  }
}

/*
 * out = P a for one Pauli string, given as one code per qubit
 * (codes[q] in {0 = I, 1 = X, 2 = Y, 3 = Z}): the tensor product is applied
 * factor by factor as single-qubit gates.
 */
void oracle_apply_pauli_string(const cplx* a, int n, const uint8_t* codes,
                               cplx* out) {
  const uint64_t N = 1ull << n;
  double q[8];
  memcpy(out, a, N * sizeof(cplx));
  for (int k = 0; k < n; k++) {
    if (codes[k] == 0) continue;
    pauli_matrix(codes[k], q);
    oracle_apply_1q(out, n, k, q);
  }
}

/*
 * <a|H|a> for H = sum_j coeff[j] P_j, codes is nterms x n (row j = P_j).
 * Each term is Re<a|P_j a> computed from the explicit product P_j a.
 * Returns 0 on success, -1 if scratch memory could not be allocated.
 */
int oracle_expect_pauli(const cplx* a, int n, int nterms, const uint8_t* codes,
                        const double* coeff, double* out) {
  const uint64_t N = 1ull << n;
  cplx* tmp = (cplx*)malloc(N * sizeof(cplx));
  if (!tmp) return -1;
  long double e = 0.0L;
  for (int j = 0; j < nterms; j++) {
    double re, im;
    oracle_apply_pauli_string(a, n, codes + (size_t)j * n, tmp);
    oracle_inner(a, tmp, n, &re, &im);
    e += (long double)coeff[j] * re;
  }
  free(tmp);
  *out = (double)e;
  return 0;
}

/*
 * out = H a = sum_j coeff[j] P_j a.  Returns 0, or -1 on allocation failure.
 */
int oracle_apply_pauli_sum(const cplx* a, int n, int nterms,
                           const uint8_t* codes, const double* coeff,
                           cplx* out) {
  const uint64_t N = 1ull << n;
  cplx* tmp = (cplx*)malloc(N * sizeof(cplx));
  if (!tmp) return -1;
  for (uint64_t i = 0; i < N; i++) out[i] = 0.0;
  for (int j = 0; j < nterms; j++) {
    oracle_apply_pauli_string(a, n, codes + (size_t)j * n, tmp);
    for (uint64_t i = 0; i < N; i++) out[i] += coeff[j] * tmp[i];
  }
  free(tmp);
  return 0;
}

/*
 * Gate list, applied in order.  The record layout is that of the circuit
 * description used throughout (80 bytes): int32 kind, target, control,
 * param; double mat[8].  Kinds: 0 = general 1-qubit gate (mat), 1 =
 * controlled gate (mat, control), 2/3/4 = RX/RY/RZ(theta[param]) with
 * R_P(theta) = exp(-i theta P / 2).
 */
typedef struct {
  int32_t kind, target, control, param;
  double mat[8];
} oracle_op;

/* The 2x2 matrix of a rotation, in the 8-double layout used above. */
void oracle_rotation_matrix(int kind, double theta, double* q) {
  const double c = cos(theta / 2.0), s = sin(theta / 2.0);
  memset(q, 0, 8 * sizeof(double));
  if (kind == 2) {        /* RX = [[c, -i s], [-i s, c]] */
    q[0] = c; q[3] = -s; q[5] = -s; q[6] = c;
  } else if (kind == 3) { /* RY = [[c, -s], [s, c]] */
    q[0] = c; q[2] = -s; q[4] = s; q[6] = c;
  } else {                /* RZ = diag(exp(-i theta/2), exp(i theta/2)) */
    q[0] = c; q[1] = -s; q[6] = c; q[7] = s;
  }
}

/* Returns 0, or -1 for an unknown kind. */
int oracle_run(cplx* a, int n, const oracle_op* ops, int nops,
               const double* theta) {
  double q[8];
  for (int g = 0; g < nops; g++) {
    const oracle_op* op = &ops[g];
    if (op->kind == 0) {
      oracle_apply_1q(a, n, op->target, op->mat);
    } else if (op->kind == 1) {
      oracle_apply_cu(a, n, op->control, op->target, op->mat);
    } else if (op->kind >= 2 && op->kind <= 4) {
      oracle_rotation_matrix(op->kind, theta[op->param], q);
      oracle_apply_1q(a, n, op->target, q);
    } else {
      return -1;
    }
  }
  return 0;
}
