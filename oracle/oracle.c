/*
 * Plain FP64 CPU oracle for the full-state operations of Jones & Benjamin,
 * "Distributed Simulation of Statevectors and Density Matrices"
 * (arXiv:2311.01512).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: every routine below is written directly from the paper's
 * definitions and local algorithms, deliberately slow and obvious.
 *
 * State layout: an N-qubit statevector is 2^N `double complex`, qubit 0 the
 * least significant index bit (Sec. "Notation").  A density matrix rho of N
 * qubits is its Choi vector of 2^(2N) entries, entry i = k + l*2^N holding
 * rho[k][l] (Sec. "State representation").
 *
 * Pins: every function here is checked by tests/test_oracle_pins.py against
 * dense Kronecker-product matrices, closed forms and invariants.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define OR_OK 0
#define OR_ERR (-1)

/* ---- bit twiddling: Alg. "bit_twiddles" ------------------------------- */

static inline uint64_t get_bit(uint64_t n, int t) { return (n >> t) & 1ULL; }

static inline uint64_t insert_bit(uint64_t n, int t, uint64_t b)
{
    uint64_t l = (n >> t) << (t + 1);
    uint64_t m = b << t;
    uint64_t r = n & ((1ULL << t) - 1ULL);
    return l | m | r;
}

/* t must be sorted increasingly */
static uint64_t insert_bits(uint64_t n, const int *t, int len, uint64_t b)
{
    for (int q = 0; q < len; q++)
        n = insert_bit(n, t[q], b);
    return n;
}

/* set bit t[q] of n to bit q of v (n holds zeros at every t[q]) */
static uint64_t set_bits(uint64_t n, const int *t, int len, uint64_t v)
{
    for (int q = 0; q < len; q++) {
        uint64_t b = get_bit(v, q) << t[q];
        n = (n & ~b) | b;
    }
    return n;
}

static uint64_t bit_mask(const int *t, int len)
{
    uint64_t m = 0;
    for (int q = 0; q < len; q++)
        m ^= 1ULL << t[q];
    return m;
}

static int parity(uint64_t x)
{
    int p = 0;
    while (x) {
        p ^= 1;
        x &= x - 1;
    }
    return p;
}

static void sort_ints(int *a, int n)
{
    for (int i = 1; i < n; i++) {
        int v = a[i], j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            j--;
        }
        a[j + 1] = v;
    }
}

/* distinct qubits in [0, N) */
static int check_qubits(const int *q, int n, int N)
{
    for (int i = 0; i < n; i++) {
        if (q[i] < 0 || q[i] >= N)
            return OR_ERR;
        for (int j = 0; j < i; j++)
            if (q[i] == q[j])
                return OR_ERR;
    }
    return OR_OK;
}

/* ---- compensated (Kahan) summation, used by every reduction ----------- */

typedef struct {
    double s, c;
} kahan;

static inline void kadd(kahan *k, double x)
{
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* ---- write counting (debug build) --------------------------------------
 * Built with -DORACLE_COUNT_WRITES, every store of a state amplitude adds
 * one to a counter, so that tests can compare each routine's writes with
 * the counts the paper states (Table "alg_summary_table" and the cost
 * statement of each algorithm's section).  The normal build compiles the
 * counting out. */
#ifdef ORACLE_COUNT_WRITES
static uint64_t g_writes;
#define WROTE(k)                      \
    do {                              \
        _Pragma("omp atomic")         \
        g_writes += (uint64_t)(k);    \
    } while (0)
#else
#define WROTE(k) \
    do {         \
    } while (0)
#endif

/* 1 when this build counts writes. */
int oracle_counts_writes(void)
{
#ifdef ORACLE_COUNT_WRITES
    return 1;
#else
    return 0;
#endif
}

/* Writes counted since the last reset (0 in the normal build). */
uint64_t oracle_writes(void)
{
#ifdef ORACLE_COUNT_WRITES
    return g_writes;
#else
    return 0;
#endif
}

void oracle_reset_writes(void)
{
#ifdef ORACLE_COUNT_WRITES
    g_writes = 0;
#endif
}

/* ---- statevector gates ------------------------------------------------ */

/*
 * Many-control many-target gate C_c(M_t): the many-target update rule
 * (Eq. "local_manyqb_amp_update"), restricted to the amplitudes that satisfy
 * the control condition (Eq. "serial_manyctrl_ctrl_cond"); controls
 * and targets are spliced into the loop index together, as Sec. "Many-target
 * gate" and Sec. "Many-control one-target gate" describe.  Matrix column /
 * row index bit q corresponds to targs[q] (in the order given), M row-major.
 */
int oracle_apply_gate(cplx *psi, int N, const int *ctrls, int nc,
                      const int *targs, int nt, const cplx *M)
{
    if (nt < 1 || nc < 0 || nc + nt > N || nc + nt > 62)
        return OR_ERR;
    int all[64];
    for (int i = 0; i < nc; i++)
        all[i] = ctrls[i];
    for (int i = 0; i < nt; i++)
        all[nc + i] = targs[i];
    if (check_qubits(all, nc + nt, N) != OR_OK)
        return OR_ERR;
    int sorted_q[64];
    memcpy(sorted_q, all, sizeof(int) * (nc + nt));
    sort_ints(sorted_q, nc + nt);

    const uint64_t ctrl_mask = bit_mask(ctrls, nc);
    const int64_t num_groups = (int64_t)(1ULL << (N - nc - nt));
    const int dim = 1 << nt;

#pragma omp parallel
    {
        cplx *v = (cplx *)malloc(sizeof(cplx) * dim); /* thread-private */
#pragma omp for schedule(static)
        for (int64_t k = 0; k < num_groups; k++) {
            uint64_t z = insert_bits((uint64_t)k, sorted_q, nc + nt, 0) | ctrl_mask;
            for (int j = 0; j < dim; j++)
                v[j] = psi[set_bits(z, targs, nt, (uint64_t)j)];
            for (int j = 0; j < dim; j++) {
                cplx acc = 0;
                for (int l = 0; l < dim; l++)
                    acc += M[(size_t)j * dim + l] * v[l];
                psi[set_bits(z, targs, nt, (uint64_t)j)] = acc;
                WROTE(1);
            }
        }
        free(v);
    }
    return OR_OK;
}

/* Pauli string masks: X/Y positions flip, Y/Z positions contribute signs
 * (Eq. "pauli_tensor_action_on_basis_state"). codes 0=I 1=X 2=Y 3=Z. */
static int pauli_masks(const int *targs, const int *paulis, int n, int N,
                       uint64_t *xy, uint64_t *yz, int *ny)
{
    if (check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    *xy = 0;
    *yz = 0;
    *ny = 0;
    for (int q = 0; q < n; q++) {
        uint64_t b = 1ULL << targs[q];
        switch (paulis[q]) {
        case 0: break;
        case 1: *xy |= b; break;
        case 2: *xy |= b; *yz |= b; (*ny)++; break;
        case 3: *yz |= b; break;
        default: return OR_ERR;
        }
    }
    return OR_OK;
}

static cplx i_pow(int k)
{
    static const cplx tab[4] = {1.0, I, -1.0, -I};
    return tab[((k % 4) + 4) % 4];
}

/* beta_x = eta * (-1)^{f(x)}, eta = i^{#Y}, f(x) = popcount(x & yz) */
static inline cplx pauli_beta(uint64_t x, uint64_t yz, cplx eta)
{
    return parity(x & yz) ? -eta : eta;
}

/*
 * Pauli gadget exp(i theta P) (Sec. "Pauli gadget"): with the Euler form
 * cos(theta) 1 + i sin(theta) P, amplitude i becomes
 * cos(theta) a_i + i sin(theta) beta_{i'} a_{i'},  i' = i with the X/Y bits
 * flipped.  Pairs (i, i') are visited once; with no X/Y this is the phase
 * gadget of Eq. "phase_gadget_amp_change".
 */
int oracle_apply_pauli_gadget(cplx *psi, int N, const int *targs,
                              const int *paulis, int n, double theta)
{
    uint64_t xy, yz;
    int ny;
    if (pauli_masks(targs, paulis, n, N, &xy, &yz, &ny) != OR_OK)
        return OR_ERR;
    const cplx eta = i_pow(ny);
    const double a = cos(theta), b = sin(theta);
    const int64_t dim = (int64_t)(1ULL << N);
    if (xy == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < dim; i++) {
            psi[i] = a * psi[i] + I * b * pauli_beta((uint64_t)i, yz, eta) * psi[i];
            WROTE(1);
        }
        return OR_OK;
    }
    int lb = 0;
    while (!((xy >> lb) & 1ULL))
        lb++;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < dim / 2; g++) {
        uint64_t i = insert_bit((uint64_t)g, lb, 0);
        uint64_t j = i ^ xy;
        cplx ai = psi[i], aj = psi[j];
        psi[i] = a * ai + I * b * pauli_beta(j, yz, eta) * aj;
        psi[j] = a * aj + I * b * pauli_beta(i, yz, eta) * ai;
        WROTE(2);
    }
    return OR_OK;
}

/*
 * SWAP gate (Sec. "Swap gate"): an amplitude whose bits t1 and t2 differ
 * takes the value of the amplitude with both bits flipped; the others keep
 * theirs.  Each changed pair is visited once, from its member with bit t1
 * set and bit t2 clear.
 */
int oracle_apply_swap(cplx *psi, int N, int t1, int t2)
{
    const int t[2] = {t1, t2};
    if (check_qubits(t, 2, N) != OR_OK)
        return OR_ERR;
    const uint64_t both = (1ULL << t1) | (1ULL << t2);
    const int64_t dim = (int64_t)(1ULL << N);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        if (get_bit((uint64_t)i, t1) == 1 && get_bit((uint64_t)i, t2) == 0) {
            const uint64_t j = (uint64_t)i ^ both;
            const cplx tmp = psi[i];
            psi[i] = psi[j];
            psi[j] = tmp;
            WROTE(2);
        }
    }
    return OR_OK;
}

/*
 * Pauli tensor (Sec. "Pauli tensor", Eq. "pauli_tensor_amp_update"):
 * amplitude i becomes beta_{i'} a_{i'}, where i' is i with every X/Y target
 * bit flipped and beta_x = eta (-1)^{f(x)}, eta = i^{#Y}, f(x) the number of
 * Y/Z targets whose bit is 1 in x.  Written out of place through a copy so
 * the update reads only old amplitudes.
 */
int oracle_apply_pauli_tensor(cplx *psi, int N, const int *targs, const int *paulis, int n)
{
    uint64_t xy, yz;
    int ny;
    if (pauli_masks(targs, paulis, n, N, &xy, &yz, &ny) != OR_OK)
        return OR_ERR;
    const cplx eta = i_pow(ny);
    const int64_t dim = (int64_t)(1ULL << N);
    cplx *old = (cplx *)malloc(sizeof(cplx) * (size_t)dim);
    if (!old)
        return OR_ERR;
    memcpy(old, psi, sizeof(cplx) * (size_t)dim);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        const uint64_t src = (uint64_t)i ^ xy;
        psi[i] = pauli_beta(src, yz, eta) * old[src];
        WROTE(1);
    }
    free(old);
    return OR_OK;
}

/*
 * Phase gadget exp(i theta Z..Z) (Sec. "Phase gadget",
 * Eq. "phase_gadget_amp_change"): amplitude i is multiplied by
 * exp(i theta s_i), s_i = +1 when an even number of the targets are 1 in i,
 * else -1.
 */
int oracle_apply_phase_gadget(cplx *psi, int N, const int *targs, int n, double theta)
{
    if (n < 1 || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    const uint64_t mask = bit_mask(targs, n);
    const int64_t dim = (int64_t)(1ULL << N);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        const double s = parity((uint64_t)i & mask) ? -1.0 : 1.0;
        psi[i] *= cexp(I * theta * s);
        WROTE(1);
    }
    return OR_OK;
}

/* ---- density matrices (Choi vectors) ---------------------------------- */

/*
 * Unitary on a density matrix (Eq. "unitary_on_vectorised_dens",
 * Alg. "distrib_dens_matr_unitary"): apply U on targets t, then conj(U)
 * on targets t+N, controls shifted alike.
 */
int oracle_dm_apply_gate(cplx *rho, int N, const int *ctrls, int nc,
                         const int *targs, int nt, const cplx *M)
{
    if (nc + nt > N || nt < 1 || nc + nt > 31)
        return OR_ERR;
    if (check_qubits(ctrls, nc, N) != OR_OK || check_qubits(targs, nt, N) != OR_OK)
        return OR_ERR;
    if (oracle_apply_gate(rho, 2 * N, ctrls, nc, targs, nt, M) != OR_OK)
        return OR_ERR;
    int c2[32], t2[32];
    for (int i = 0; i < nc; i++)
        c2[i] = ctrls[i] + N;
    for (int i = 0; i < nt; i++)
        t2[i] = targs[i] + N;
    const int dim = 1 << nt;
    cplx *Mc = (cplx *)malloc(sizeof(cplx) * dim * dim);
    for (int i = 0; i < dim * dim; i++)
        Mc[i] = conj(M[i]);
    int r = oracle_apply_gate(rho, 2 * N, c2, nc, t2, nt, Mc);
    free(Mc);
    return r;
}

/*
 * Pauli gadget on a density matrix (Alg. "distrib_dens_matr_specific_unitaries"):
 * the gadget on t with theta, then on t+N with theta negated once, and once
 * more per Y operator, since conj(exp(i theta P)) = exp(i (-1)^{m+1} theta P)
 * for m Y operators.
 */
int oracle_dm_apply_pauli_gadget(cplx *rho, int N, const int *targs,
                                 const int *paulis, int n, double theta)
{
    if (n > 32 || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    if (oracle_apply_pauli_gadget(rho, 2 * N, targs, paulis, n, theta) != OR_OK)
        return OR_ERR;
    int t2[64];
    double th = -theta;
    for (int q = 0; q < n; q++) {
        t2[q] = targs[q] + N;
        if (paulis[q] == 2)
            th = -th;
    }
    return oracle_apply_pauli_gadget(rho, 2 * N, t2, paulis, n, th);
}

/*
 * SWAP, Pauli tensor and phase gadget on a density matrix
 * (Alg. "distrib_dens_matr_specific_unitaries"), each the statevector
 * routine on the Choi vector twice, using conj(SWAP) = SWAP,
 * conj(P) = (-1)^m P for m Y operators, and
 * conj(exp(i theta Z..Z)) = exp(-i theta Z..Z).
 */
int oracle_dm_apply_swap(cplx *rho, int N, int t1, int t2)
{
    const int t[2] = {t1, t2};
    if (check_qubits(t, 2, N) != OR_OK)
        return OR_ERR;
    if (oracle_apply_swap(rho, 2 * N, t1, t2) != OR_OK)
        return OR_ERR;
    return oracle_apply_swap(rho, 2 * N, t1 + N, t2 + N);
}

int oracle_dm_apply_pauli_tensor(cplx *rho, int N, const int *targs, const int *paulis, int n)
{
    if (n > 32 || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    if (oracle_apply_pauli_tensor(rho, 2 * N, targs, paulis, n) != OR_OK)
        return OR_ERR;
    int t2[64];
    int m = 0;
    for (int q = 0; q < n; q++) {
        t2[q] = targs[q] + N;
        if (paulis[q] == 2)
            m = !m;
    }
    if (oracle_apply_pauli_tensor(rho, 2 * N, t2, paulis, n) != OR_OK)
        return OR_ERR;
    if (m) {
        const int64_t dim = (int64_t)(1ULL << (2 * N));
        for (int64_t j = 0; j < dim; j++)
            rho[j] *= -1.0;
    }
    return OR_OK;
}

int oracle_dm_apply_phase_gadget(cplx *rho, int N, const int *targs, int n, double theta)
{
    if (n < 1 || n > 32 || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    if (oracle_apply_phase_gadget(rho, 2 * N, targs, n, theta) != OR_OK)
        return OR_ERR;
    int t2[64];
    for (int q = 0; q < n; q++)
        t2[q] = targs[q] + N;
    return oracle_apply_phase_gadget(rho, 2 * N, t2, n, -theta);
}

/*
 * Superoperator of a Kraus map (Eq. "superop_from_kraus_map",
 * Alg. "distrib_dens_matr_kraus_map"):
 * S[i 2^n + k][j 2^n + l] = sum_m conj(K_m[i][j]) K_m[k][l].
 * K is M consecutive row-major 2^n x 2^n matrices; S is row-major 4^n x 4^n.
 */
int oracle_build_superop(const cplx *K, int num_ops, int n, cplx *S)
{
    if (n < 1 || n > 6 || num_ops < 1)
        return OR_ERR;
    const int d = 1 << n, D = d * d;
    memset(S, 0, sizeof(cplx) * (size_t)D * D);
    for (int m = 0; m < num_ops; m++) {
        const cplx *Km = K + (size_t)m * D;
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++)
                for (int k = 0; k < d; k++)
                    for (int l = 0; l < d; l++) {
                        int r = i * d + k, c = j * d + l;
                        S[(size_t)r * D + c] += conj(Km[i * d + j]) * Km[k * d + l];
                    }
    }
    return OR_OK;
}

/* Superoperator S on targets t of a density matrix: the 2n-target gate S on
 * the Choi vector with targets t' = (t_0..t_{n-1}, t_0+N..t_{n-1}+N). */
int oracle_dm_apply_superop(cplx *rho, int N, const int *targs, int n, const cplx *S)
{
    if (n < 1 || 2 * n > 2 * N || n > 16 || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    int t2[32];
    for (int q = 0; q < n; q++) {
        t2[q] = targs[q];
        t2[q + n] = targs[q] + N;
    }
    return oracle_apply_gate(rho, 2 * N, NULL, 0, t2, 2 * n, S);
}

int oracle_dm_apply_kraus(cplx *rho, int N, const int *targs, int n,
                          const cplx *K, int num_ops)
{
    if (n < 1 || n > 6)
        return OR_ERR;
    const size_t D = (size_t)1 << (2 * n);
    cplx *S = (cplx *)malloc(sizeof(cplx) * D * D);
    int r = oracle_build_superop(K, num_ops, n, S);
    if (r == OR_OK)
        r = oracle_dm_apply_superop(rho, N, targs, n, S);
    free(S);
    return r;
}

/*
 * Partial trace (Eq. "partial_trace_reduced_amp_def", Alg. "distrib_partial_trace"
 * local subroutine): output entry i of the (N-n)-qubit Choi vector is the sum
 * over v < 2^n of input entry g(i, v), g splicing the bits of v in at the
 * positions t and again at t+N.  Outputs are iterated, inputs gathered.
 */
int oracle_partial_trace(const cplx *rho, int N, const int *targs, int n, cplx *out)
{
    if (n < 1 || n >= N || check_qubits(targs, n, N) != OR_OK)
        return OR_ERR;
    int t2[64], s[128];
    for (int q = 0; q < n; q++) {
        t2[q] = targs[q] + N;
        s[q] = targs[q];
        s[q + n] = t2[q];
    }
    sort_ints(s, 2 * n);
    const int64_t out_len = (int64_t)(1ULL << (2 * (N - n)));
    const uint64_t nv = 1ULL << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < out_len; i++) {
        uint64_t g0 = insert_bits((uint64_t)i, s, 2 * n, 0);
        kahan re = {0, 0}, im = {0, 0};
        for (uint64_t v = 0; v < nv; v++) {
            uint64_t g = set_bits(g0, targs, n, v);
            g = set_bits(g, t2, n, v);
            kadd(&re, creal(rho[g]));
            kadd(&im, cimag(rho[g]));
        }
        out[i] = re.s + I * im.s;
        WROTE(1);
    }
    return OR_OK;
}

/* ---- calculations ------------------------------------------------------ */

/*
 * Pauli-sum expectation of a density matrix (Eq. "dens_expec_val_sum",
 * Alg. "distrib_dens_matr_pauli_string_expec"): sum_i H_i beta_i with
 * H_i = sum_n h_n prod_q sigma_q^{(n)}[i_{q+N}, i_q].  codes is T*N,
 * term-major then qubit 0 first.  Every entry is visited (the paper's
 * algorithm); the result is complex.
 */
int oracle_dm_expec_pauli_sum(const cplx *rho, int N, const int *codes,
                              const double *coeffs, int T, double *out_re, double *out_im)
{
    static const cplx P[4][2][2] = {
        {{1, 0}, {0, 1}},
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    const uint64_t len = 1ULL << (2 * N);
    kahan re = {0, 0}, im = {0, 0};
    for (uint64_t i = 0; i < len; i++) {
        cplx h = 0;
        for (int t = 0; t < T; t++) {
            cplx v = 1;
            for (int q = 0; q < N; q++) {
                int bc = (int)get_bit(i, q), br = (int)get_bit(i, q + N);
                v *= P[codes[t * N + q]][br][bc];
            }
            h += coeffs[t] * v;
        }
        cplx x = h * rho[i];
        kadd(&re, creal(x));
        kadd(&im, cimag(x));
    }
    *out_re = re.s;
    *out_im = im.s;
    return OR_OK;
}

/*
 * Pauli-sum expectation of a statevector, from the definition
 * <psi|H|psi> = sum_n h_n sum_i conj(a_i) (P_n psi)_i, where P_n acts by
 * Eq. "pauli_tensor_amp_update": (P psi)_i = beta_{i'} a_{i'}.
 */
int oracle_sv_expec_pauli_sum(const cplx *psi, int N, const int *codes,
                              const double *coeffs, int T, double *out_re, double *out_im)
{
    const uint64_t len = 1ULL << N;
    kahan re = {0, 0}, im = {0, 0};
    int targs[64];
    for (int q = 0; q < N; q++)
        targs[q] = q;
    for (int t = 0; t < T; t++) {
        uint64_t xy, yz;
        int ny;
        if (pauli_masks(targs, codes + (size_t)t * N, N, N, &xy, &yz, &ny) != OR_OK)
            return OR_ERR;
        const cplx eta = i_pow(ny);
        for (uint64_t i = 0; i < len; i++) {
            uint64_t j = i ^ xy;
            cplx x = coeffs[t] * conj(psi[i]) * pauli_beta(j, yz, eta) * psi[j];
            kadd(&re, creal(x));
            kadd(&im, cimag(x));
        }
    }
    *out_re = re.s;
    *out_im = im.s;
    return OR_OK;
}

/* Born rule: P(qubit q = b) = sum over i with i_q = b of |a_i|^2. */
int oracle_sv_prob_of_outcome(const cplx *psi, int N, int q, int b, double *out)
{
    if (q < 0 || q >= N || (b != 0 && b != 1))
        return OR_ERR;
    kahan s = {0, 0};
    for (uint64_t i = 0; i < (1ULL << N); i++)
        if ((int)get_bit(i, q) == b)
            kadd(&s, creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]));
    *out = s.s;
    return OR_OK;
}

/* Density matrix: P(q = b) = sum over k with k_q = b of Re rho[k][k], the
 * diagonal sitting at Choi index k (2^N + 1). */
int oracle_dm_prob_of_outcome(const cplx *rho, int N, int q, int b, double *out)
{
    if (q < 0 || q >= N || (b != 0 && b != 1))
        return OR_ERR;
    kahan s = {0, 0};
    const uint64_t stride = (1ULL << N) + 1ULL;
    for (uint64_t k = 0; k < (1ULL << N); k++)
        if ((int)get_bit(k, q) == b)
            kadd(&s, creal(rho[k * stride]));
    *out = s.s;
    return OR_OK;
}

int oracle_sv_total_prob(const cplx *psi, int N, double *out)
{
    kahan s = {0, 0};
    for (uint64_t i = 0; i < (1ULL << N); i++)
        kadd(&s, creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]));
    *out = s.s;
    return OR_OK;
}

/* Tr(rho) = sum_j beta_{j (2^N + 1)} (Sec. "Pauli string expectation value"). */
int oracle_dm_trace(const cplx *rho, int N, double *out_re, double *out_im)
{
    kahan re = {0, 0}, im = {0, 0};
    const uint64_t stride = (1ULL << N) + 1ULL;
    for (uint64_t k = 0; k < (1ULL << N); k++) {
        kadd(&re, creal(rho[k * stride]));
        kadd(&im, cimag(rho[k * stride]));
    }
    *out_re = re.s;
    *out_im = im.s;
    return OR_OK;
}

/* Tr(rho^2) = sum_{k,l} rho[k][l] rho[l][k], no Hermiticity assumed. */
int oracle_dm_purity(const cplx *rho, int N, double *out_re, double *out_im)
{
    kahan re = {0, 0}, im = {0, 0};
    const uint64_t d = 1ULL << N;
    for (uint64_t l = 0; l < d; l++)
        for (uint64_t k = 0; k < d; k++) {
            cplx x = rho[k + l * d] * rho[l + k * d];
            kadd(&re, creal(x));
            kadd(&im, cimag(x));
        }
    *out_re = re.s;
    *out_im = im.s;
    return OR_OK;
}

/* ---- canonical states (Sec. "State representation") ------------------- */

int oracle_init_basis(cplx *psi, int num_index_bits, uint64_t index)
{
    const uint64_t len = 1ULL << num_index_bits;
    if (index >= len)
        return OR_ERR;
    memset(psi, 0, sizeof(cplx) * len);
    psi[index] = 1.0;
    return OR_OK;
}

/* |+><+| of N qubits: every entry 1/2^N (the uniform state's outer product). */
int oracle_init_plus(cplx *psi, int N, int is_density)
{
    const uint64_t len = 1ULL << (is_density ? 2 * N : N);
    const double v = is_density ? ldexp(1.0, -N) : 1.0 / sqrt((double)(1ULL << N));
    for (uint64_t i = 0; i < len; i++)
        psi[i] = v;
    return OR_OK;
}

/* |psi><psi|: Choi entry j + k 2^N = psi_j conj(psi_k). */
int oracle_init_pure_dm(cplx *rho, const cplx *psi, int N)
{
    const uint64_t d = 1ULL << N;
    for (uint64_t k = 0; k < d; k++)
        for (uint64_t j = 0; j < d; j++)
            rho[j + k * d] = psi[j] * conj(psi[k]);
    return OR_OK;
}

/*
 * Counter-based "hashed" state: entry i = (u(2i) + i u(2i+1)) * 2^-ceil(L/2)
 * with u(c) = 2 * top53(splitmix64(seed + (c+1) * golden)) * 2^-53 - 1,
 * SplitMix64 as published by Steele, Lea & Flood (OOPSLA 2014).  L is the
 * number of index bits (N, or 2N for a density matrix).  The same definition
 * is implemented independently on the GPU side, so inputs of any size can be
 * regenerated amplitude by amplitude here.
 */
static uint64_t splitmix64_at(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double hashed_unit(uint64_t seed, uint64_t counter)
{
    return 2.0 * ldexp((double)(splitmix64_at(seed, counter) >> 11), -53) - 1.0;
}

uint64_t oracle_splitmix64_at(uint64_t seed, uint64_t counter)
{
    return splitmix64_at(seed, counter);
}

/* entries [start, start+count) of the hashed state with L index bits */
int oracle_hashed_amps(int L, uint64_t seed, uint64_t start, uint64_t count, cplx *out)
{
    const int e = (L + 1) / 2;
    for (uint64_t c = 0; c < count; c++) {
        uint64_t i = start + c;
        out[c] = ldexp(hashed_unit(seed, 2 * i), -e) + I * ldexp(hashed_unit(seed, 2 * i + 1), -e);
    }
    return OR_OK;
}

int oracle_hashed_amps_at(int L, uint64_t seed, const uint64_t *idx, uint64_t count, cplx *out)
{
    const int e = (L + 1) / 2;
    for (uint64_t c = 0; c < count; c++) {
        uint64_t i = idx[c];
        out[c] = ldexp(hashed_unit(seed, 2 * i), -e) + I * ldexp(hashed_unit(seed, 2 * i + 1), -e);
    }
    return OR_OK;
}

/* Threads the oracle's parallel loops use (for reporting). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
