/*
 * qsim.h — C ABI of the MI355X (gfx950) full-state simulator.
 *
 * Operations follow Jones & Benjamin, "Distributed Simulation of Statevectors
 * and Density Matrices" (arXiv:2311.01512); each declaration cites the section
 * or equation that defines what it computes.  On one GPU the whole state is
 * local, so every operation is the paper's local (non-exchanging) case.
 *
 * Conventions
 *  - Qubit 0 is the least significant bit of an amplitude index
 *    (Sec. "Notation").
 *  - A statevector of N qubits holds 2^N complex amplitudes.  A density
 *    matrix of N qubits is held as its Choi vector of 2^(2N) amplitudes,
 *    entry k + l*2^N = rho[k][l] (Sec. "State representation").
 *  - Amplitudes in device memory are interleaved (re, im) pairs of float
 *    (QS_C64) or double (QS_C128).
 *  - Host-side matrices are row-major interleaved (re, im) doubles.  For a
 *    gate on targets t[0..n-1], bit q of a matrix row/column index belongs to
 *    target t[q] (Sec. "Many-target gate").  Matrices need not be unitary, nor
 *    Kraus maps trace preserving.
 *  - Pauli codes: 0 = I, 1 = X, 2 = Y, 3 = Z.
 *  - Every call returns a status (QS_OK = 0 or a negative QS_E_* code); on
 *    failure nothing is modified and qs_last_error() describes the problem.
 *    No exception crosses this boundary.
 *  - Calls that update a state are asynchronous on the qureg's HIP stream.
 *    Calls that return a scalar synchronise that stream before returning.
 *  - Host arrays passed in are read during the call only; the caller keeps
 *    ownership.  Calls on one qureg must not run concurrently from several
 *    host threads.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_qureg qs_qureg;
typedef struct qs_circuit qs_circuit;

enum { QS_C64 = 0, QS_C128 = 1 };

enum {
    QS_OK = 0,
    QS_E_ARG = -1,     /* malformed argument (qubit out of range, duplicate, bad size) */
    QS_E_PRECOND = -2, /* operation not valid for this qureg (e.g. density-only op on a statevector) */
    QS_E_ALLOC = -3,   /* device or host allocation failed */
    QS_E_HIP = -4,     /* a HIP runtime call failed */
    QS_E_TYPE = -5     /* precision mismatch between quregs */
};

/* ---- quregs ------------------------------------------------------------ */

/*
 * Create a statevector (is_density = 0, 2^N amplitudes) or density matrix
 * (is_density = 1, Choi vector of 2^(2N) amplitudes) of num_qubits qubits.
 * device_ptr: NULL to let the library allocate (and later free) the
 * amplitudes; otherwise a device buffer of at least 2^(N or 2N) amplitudes of
 * the given precision that the caller owns and keeps alive until
 * qs_destroy_qureg.  hip_stream: the hipStream_t all work on this qureg is
 * ordered on (NULL = the null stream).  The state is not initialised.
 * Sizes: 1 <= num_qubits, and the amplitude count must fit in device memory.
 */
int qs_create_qureg(int num_qubits, int is_density, int precision,
                    void *device_ptr, void *hip_stream, qs_qureg **out);

/* Free the qureg and, if the library allocated them, its amplitudes. */
int qs_destroy_qureg(qs_qureg *q);

/* Shape of a qureg; any output pointer may be NULL. */
int qs_get_info(const qs_qureg *q, int *num_qubits, int *is_density,
                int *precision, uint64_t *num_amps, void **device_ptr);

/* Change the stream the qureg's work is ordered on (NULL = null stream). */
int qs_set_stream(qs_qureg *q, void *hip_stream);

/* Block until all work queued on the qureg's stream is done. */
int qs_sync(qs_qureg *q);

/* Thread-local description of the last failed call on this thread. */
const char *qs_last_error(void);

/* ---- initial states (Sec. "State representation") ------------------------ */

/* |0..0>, or |0><0| for a density matrix. */
int qs_init_zero_state(qs_qureg *q);

/* |i>, or |i><i| (Choi entry i (2^N + 1)) for a density matrix; i < 2^N. */
int qs_init_basis_state(qs_qureg *q, uint64_t index);

/* |+..+>: every amplitude 2^(-N/2); for a density matrix every entry 2^-N. */
int qs_init_plus_state(qs_qureg *q);

/* rho = |psi><psi|: Choi entry j + k 2^N = psi_j conj(psi_k).  rho must be a
 * density matrix and psi a statevector of the same size and precision. */
int qs_init_pure_density(qs_qureg *rho, const qs_qureg *psi);

/*
 * Unnormalised pseudo-random state from a counter-based generator, defined
 * entry by entry so that any entry can be regenerated independently:
 * entry i = (u(2i) + i u(2i+1)) * 2^-ceil(L/2), L = number of index bits
 * (N, or 2N for a density matrix), u(c) = 2 * (x >> 11) * 2^-53 - 1 with
 * x = SplitMix64 output number c of a generator seeded with `seed`
 * (Steele, Lea & Flood, OOPSLA 2014).  QS_C64 rounds the FP64 value to float.
 */
int qs_init_hashed_state(qs_qureg *q, uint64_t seed);

/* Copy count amplitudes starting at index start between the device and a
 * host array of 2*count doubles (re, im interleaved).  Synchronous. */
int qs_set_amps(qs_qureg *q, uint64_t start, const double *re_im, uint64_t count);
int qs_get_amps(const qs_qureg *q, uint64_t start, double *re_im, uint64_t count);

/* ---- operators ------------------------------------------------------------ */

/*
 * Many-control many-target gate C_ctrls(M_targs) (Sec. "Many-control
 * one-target gate", Eq. "serial_manyctrl_ctrl_cond"; Sec. "Many-target gate",
 * Eq. "local_manyqb_amp_update"): every amplitude whose control bits are all 1
 * is replaced by the matrix-weighted combination of the 2^n amplitudes that
 * differ from it only on the targets; the others are untouched.  matrix is
 * 2^n x 2^n (n = num_targs, 1 <= n <= 6), row-major (re, im) doubles.
 * Controls and targets must be distinct qubits < N.  On a density matrix it
 * applies rho -> U rho U^dagger (Eq. "unitary_on_vectorised_dens": U on the
 * targets, conj(U) on the targets shifted by N, controls shifted alike).
 */
int qs_apply_multi_ctrl_multi_targ_unitary(qs_qureg *q, const int *ctrls, int num_ctrls,
                                           const int *targs, int num_targs,
                                           const double *matrix);

/*
 * Pauli gadget exp(i theta P), P = tensor of paulis[q] on targs[q]
 * (Sec. "Pauli gadget"; Sec. "Phase gadget" when P has no X or Y).  Codes
 * 0..3; identity entries are ignored.  On a density matrix it applies
 * rho -> G rho G^dagger: the gadget on the targets and, with angle
 * (-1)^(m+1) theta (m = number of Y), on the targets shifted by N
 * (Alg. "distrib_dens_matr_specific_unitaries"), fused into one pass over
 * the Choi vector.  Targets distinct and < N (QS_E_ARG).
 */
int qs_apply_pauli_gadget(qs_qureg *q, const int *targs, const int *paulis,
                          int num_targs, double theta);

/*
 * SWAP gate on qubits qubit1 != qubit2 (Sec. "Swap gate"): amplitudes whose
 * two bits differ trade places with the amplitude that has both bits
 * flipped; no floating-point work, and only the moved half of the state is
 * written.  On a density matrix, rho -> SWAP rho SWAP: the same swap on the
 * column bits t + N, since conj(SWAP) = SWAP (Alg.
 * "distrib_dens_matr_specific_unitaries"), in the same pass.
 * Qubits distinct and < N (QS_E_ARG).  Asynchronous on the qureg's stream.
 */
int qs_apply_swap(qs_qureg *q, int qubit1, int qubit2);

/*
 * num_pairs disjoint SWAPs (qubits1[k], qubits2[k]) at once: the qubit
 * remapping that moves a many-target gate's high targets onto low qubits
 * (Sec. "Many-target gate", the SWAP conjugation of an upper-targeting
 * gate).  Up to 3 index-bit pairs share a pass (a density matrix counts
 * each pair twice).  All 2 num_pairs qubits distinct and < N (QS_E_ARG).
 */
int qs_apply_multi_swap(qs_qureg *q, const int *qubits1, const int *qubits2, int num_pairs);

/*
 * Pauli tensor P = tensor of paulis[q] (codes 0..3) on targs[q]
 * (Sec. "Pauli tensor", Eq. "pauli_tensor_amp_update"): amplitude i becomes
 * beta a_{i'}, i' = i with the X/Y target bits flipped, beta a unit
 * (+-1, +-i) fixed by i' and the Y/Z targets; one pass, no products.  On a
 * density matrix, rho -> P rho P^dagger: P on the targets and
 * conj(P) = (-1)^m P on the targets shifted by N (Eq.
 * "distrib_pauli_tensor_conj"), one pass.  Targets distinct and < N,
 * codes in 0..3 (QS_E_ARG).
 */
int qs_apply_pauli_tensor(qs_qureg *q, const int *targs, const int *paulis, int num_targs);

/*
 * Phase gadget exp(i theta Z (x) ... (x) Z) on targs (Sec. "Phase gadget",
 * Eq. "phase_gadget_amp_change"): amplitude i is multiplied by
 * exp(i theta s_i), s_i = -1 when an odd number of the targets are 1 in i,
 * else +1.  On a density matrix, exp(i theta Z..Z) on the targets and
 * exp(-i theta Z..Z) on the targets shifted by N, one diagonal pass.
 * Targets distinct and < N (QS_E_ARG).
 */
int qs_apply_phase_gadget(qs_qureg *q, const int *targs, int num_targs, double theta);

/*
 * Superoperator S (4^n x 4^n, row-major (re, im) doubles) on targets t of a
 * density matrix: the 2n-target gate S on the Choi vector with targets
 * (t[0]..t[n-1], t[0]+N..t[n-1]+N) (Sec. "Kraus map", Alg.
 * "distrib_dens_matr_kraus_map").  1 <= n <= 3.  Density matrices only.
 */
int qs_apply_superop(qs_qureg *q, const int *targs, int num_targs, const double *superop);

/*
 * Kraus map rho -> sum_m K_m rho K_m^dagger (Sec. "Kraus map"): builds
 * S = sum_m conj(K_m) (x) K_m in FP64 on the host
 * (Eq. "superop_from_kraus_map") and applies it as qs_apply_superop.
 * kraus holds num_ops consecutive 2^n x 2^n row-major (re, im) matrices.
 * 1 <= n <= 3, num_ops >= 1.  Density matrices only.
 */
int qs_apply_kraus_map(qs_qureg *q, const int *targs, int num_targs,
                       const double *kraus, int num_ops);

/*
 * Decoherence channels on a density matrix, each one pass over the Choi
 * vector with the channel's closed-form update (no superoperator):
 *   dephasing, prob. p (Sec. "dephasing", Alg.
 *     "distrib_dens_matr_one_qb_dephasing"): rho -> (1-p) rho + p Z rho Z,
 *     i.e. beta_i -> (1 - 2p) beta_i where bits t and t+N of i differ; the
 *     other half of the state is not touched;
 *   two-qubit dephasing (Eq. "dephasing_2qb_update_rule", Alg.
 *     "distrib_dens_matr_two_qb_dephasing"): Z on t1, t2 or both with total
 *     prob. p; beta_i -> (1 - 4p/3) beta_i unless both principal pairs agree
 *     (those three quarters only are read and written);
 *   depolarising, total prob. p, p/3 per Pauli (Eq.
 *     "depolarising_1qb_amp_update", Alg. "distrib_dens_matr_one_qb_depolarising");
 *   two-qubit depolarising, total prob. p, p/15 per non-identity Pauli pair
 *     (Eq. "2qb_depolarising_choi_amp_update", Alg.
 *     "distrib_dens_matr_two_qb_depolarising");
 *   amplitude damping, decay prob. p (Eq. "damping_amps_update", Alg.
 *     "distrib_dens_matr_damping").
 * 0 <= p <= 1 (QS_E_ARG otherwise); targets distinct and < N (QS_E_ARG);
 * density matrices only (QS_E_PRECOND).  Asynchronous on the qureg's stream.
 */
int qs_apply_dephasing(qs_qureg *q, int target, double p);
int qs_apply_two_qubit_dephasing(qs_qureg *q, int target1, int target2, double p);
int qs_apply_depolarising(qs_qureg *q, int target, double p);
int qs_apply_two_qubit_depolarising(qs_qureg *q, int target1, int target2, double p);
int qs_apply_damping(qs_qureg *q, int target, double p);

/* ---- calculations ---------------------------------------------------------- */

/*
 * Partial trace over targs (Sec. "Partial trace", Eq.
 * "partial_trace_reduced_amp_def"): out[i] = sum_{v < 2^n} in[g(i, v)],
 * g splicing the bits of v in at the traced qubits and again at those
 * qubits + N.  The kept qubits keep their relative order.  in and out are
 * density matrices of the same precision, out has N - n qubits, 1 <= n < N.
 * Asynchronous on in's stream; out is ordered after it.
 */
int qs_calc_partial_trace(const qs_qureg *in, const int *targs, int num_targs, qs_qureg *out);

/*
 * Expectation of H = sum_t coeffs[t] (x)_q P(paulis[t*N + q]) (Sec. "Pauli
 * string expectation value").  paulis: num_terms * N codes, term-major then
 * qubit 0 first.  Density matrix: Tr(H rho) (Eq. "dens_expec_val_sum").
 * Statevector: <psi|H|psi>.  On 8 or more qubits the terms are grouped
 * into spans of up to 7 X/Y flip masks beyond the 4 lowest qubits, and the
 * state is read once per span (tiles held on chip); each term sums its real
 * or its imaginary part, whichever a Hermitian string can give, so *out_im
 * is exactly 0 there.  Accumulated in FP64 in a fixed order (repeated calls
 * give identical results); *out_im is the imaginary part (zero up to
 * rounding for Hermitian rho).  Either output may be NULL.  Blocks until
 * the value is on the host.
 */
int qs_calc_expec_pauli_sum(const qs_qureg *q, const int *paulis, const double *coeffs,
                            int num_terms, double *out_re, double *out_im);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the value
 * of qs_calc_expec_pauli_sum computed on a caller's device buffer with no
 * qureg and no allocation of any kind.  amps: device pointer of the current
 * device holding 2^num_qubits (statevector) or 2^(2 num_qubits) (density
 * matrix, Choi vector) interleaved amplitudes of the given precision,
 * owned by the caller; hip_stream: the hipStream_t the work is ordered on
 * (NULL = null stream).  paulis, coeffs, num_terms, out_re, out_im as for
 * qs_calc_expec_pauli_sum; the result and its summation order are the same.
 * Scratch: a library-owned static device array of 256 KiB + 512 B per GPU,
 * which every size fits (the reductions cap their partial sums), kept until
 * the process ends.  All calls on one GPU share it: calls that overlap on
 * one GPU race.  Errors: QS_E_ARG for a null or non-device pointer, memory
 * of another device, a bad precision or qubit count (index bits <= 62), or
 * a malformed Pauli sum; QS_E_HIP if a HIP call fails.  Blocks until the
 * value is on the host.
 */
int qs_calc_expec_pauli_sum_noalloc(const void *amps, int num_qubits, int is_density, int precision,
                                    void *hip_stream, const int *paulis, const double *coeffs,
                                    int num_terms, double *out_re, double *out_im);

/* Probability that measuring `qubit` gives `outcome` (0/1): the sum of |a_i|^2
 * over i with that bit (Born rule), or of Re rho[k][k] for a density matrix.
 * Not renormalised.  FP64 accumulation. */
int qs_calc_prob_of_outcome(const qs_qureg *q, int qubit, int outcome, double *out);

/* Statevector: sum |a_i|^2.  Density matrix: Re Tr(rho). */
int qs_calc_total_prob(const qs_qureg *q, double *out);

/* Density matrix: Tr(rho) as (re, im) (Sec. "Pauli string expectation value",
 * trace of a Choi vector). */
int qs_calc_trace(const qs_qureg *q, double *out_re, double *out_im);

/* Density matrix: Tr(rho^2) = sum_{k,l} rho[k][l] rho[l][k] as (re, im). */
int qs_calc_purity(const qs_qureg *q, double *out_re, double *out_im);

/* Statevector: <a|b> = sum conj(a_i) b_i, FP64 accumulation. */
int qs_calc_inner_product(const qs_qureg *a, const qs_qureg *b, double *out_re, double *out_im);

/* ---- circuits: recorded op lists, optionally fused into dense blocks ------- */

/*
 * A circuit records operators for later application.  A statevector
 * circuit holds gates and Pauli gadgets on N qubits; a density circuit
 * (qs_circuit_create_density) holds them for an N-qubit density matrix and
 * records each as the Choi-vector operators of Sec. "density matrices"
 * (U on the row qubits t, conj(U) on the column qubits t + N; a gadget on t
 * and again on t + N with the conjugate's angle), plus superoperators and
 * Kraus maps on (t, t + N).  Compiling plans passes over the 2N index bits.
 *
 * fuse_k = 0 keeps one pass per operator (the plain per-gate method).
 * 2 <= fuse_k <= 6 merges operators into dense blocks of at most fuse_k
 * qubits: an operator joins the current block when the block's qubit set
 * stays within fuse_k qubits and the operator commutes with every operator
 * it is moved across (disjoint qubits).  A block's matrix is the FP64
 * product of its members, each written densely on the block's qubits
 * (controls expanded, a gadget as cos(theta) 1 + i sin(theta) P, Sec.
 * "Pauli gadget").  Operators on more than fuse_k qubits stay single passes.
 * Blocks of 4-6 qubits on complex64 run as FP32 MFMA GEMMs.
 * 8 <= fuse_k <= 13 plans tile steps of at most 2^fuse_k amplitudes (a
 * coset of a GF(2) subspace of the index space holding the lowest qubits,
 * every target of a member gate and every gadget's X/Y flip mask): each
 * step reads the state once, applies all its members on chip, and writes it
 * once.  Gates of up to 3 targets (complex64: 4, on the matrix cores) and
 * 4 controls, and gadgets of any weight, join steps; other operators stay
 * single passes.  The largest fuse_k a device allows depends on its LDS per
 * block (2^fuse_k amplitudes).
 *
 * The circuit owns device copies of its matrices for one precision; it must
 * outlive the work queued by qs_apply_circuit.
 */
int qs_circuit_create(int num_qubits, qs_circuit **out);
/* Density circuit for an N-qubit density matrix, 1 <= N <= 20. */
int qs_circuit_create_density(int num_qubits, qs_circuit **out);
int qs_circuit_destroy(qs_circuit *c);
/* Same arguments and meaning as qs_apply_multi_ctrl_multi_targ_unitary. */
int qs_circuit_add_unitary(qs_circuit *c, const int *ctrls, int num_ctrls, const int *targs, int num_targs,
                           const double *matrix);
/* Same arguments and meaning as qs_apply_pauli_gadget. */
int qs_circuit_add_pauli_gadget(qs_circuit *c, const int *targs, const int *paulis, int num_targs, double theta);
/* Density circuits only (QS_E_PRECOND otherwise); same arguments and
 * meaning as qs_apply_superop and qs_apply_kraus_map (the Kraus map is
 * stored as its superoperator, built in FP64). */
int qs_circuit_add_superop(qs_circuit *c, const int *targs, int num_targs, const double *superop);
int qs_circuit_add_kraus_map(qs_circuit *c, const int *targs, int num_targs, const double *kraus, int num_ops);
/* Builds the pass list (see above); precision selects the device matrix
 * layout.  QS_E_ARG for a fuse_k outside 0, 2..6, 8..13 or beyond the
 * device's tile limit. */
int qs_circuit_compile(qs_circuit *c, int fuse_k, int precision);

/*
 * Run-time specialisation of a compiled circuit's tile steps: each step
 * becomes a kernel of its own, generated as HIP source with the step's
 * register phases and operators as compile-time constants and compiled for
 * the current device by `$ROCM_PATH/llvm/bin/clang++` (default /opt/rocm),
 * run as up to eight child processes with sources written to a temporary
 * directory under $TMPDIR (default /tmp) that is removed afterwards (seconds
 * for hundreds of operators; code objects are cached per source for the
 * process, and on disk in $QS_JIT_CACHE, default $TMPDIR/qs_jit_cache, used
 * only if that directory belongs to the calling user and is not writable by
 * others).  Applying the circuit then
 * launches these kernels; results equal those of the generic tile kernel.
 * *num_kernels (may be NULL) receives the number of specialised steps (0 for
 * a circuit without tile steps).  Recompiling or destroying the circuit
 * releases them.  Errors: QS_E_PRECOND if not compiled, QS_E_HIP if the
 * run-time compilation or module load fails (the circuit keeps the generic
 * kernels).
 */
int qs_circuit_specialize(qs_circuit *c, int *num_kernels);
/* Pass statistics of the compiled circuit; any pointer may be NULL.
 * logical_updates: amplitude updates under the plain per-gate accounting
 * (2^(N-s) per s-controlled gate, 2^N per gadget) of the recorded ops;
 * blocks_by_width: array of 7 counters, passes by number of qubits (index
 * 0 counts single gadget passes). */
int qs_circuit_stats(const qs_circuit *c, int *num_ops, int *num_passes, uint64_t *logical_updates,
                     int *blocks_by_width);
/* Applies the compiled circuit to a qureg of the circuit's size, kind
 * (statevector or density matrix) and compiled precision, in order, on the
 * qureg's stream. */
int qs_apply_circuit(qs_qureg *q, qs_circuit *c);

/* Applies passes [first, first + count) of the compiled circuit (same rules
 * as qs_apply_circuit); lets a caller time passes one by one. */
int qs_apply_circuit_passes(qs_qureg *q, qs_circuit *c, int first, int count);

/* Describes pass `index` of the compiled circuit: kernel = 0 Pauli-gadget
 * pairs, 1 phase gadget (diagonal), 2 dense gate on vector FMAs, 3 dense
 * gate on FP32 MFMA, 4 tile step; num_targs / num_ctrls of a dense pass
 * (gadget: its Pauli count, 0; tile step: its dimension, 0); members =
 * recorded ops merged into the pass; phases = register layouts a tile step
 * moves through (1 for other passes).  Any out pointer may be NULL. */
int qs_circuit_pass_info(const qs_circuit *c, int index, int *kernel, int *num_targs, int *num_ctrls,
                         int *members, int *phases);

/*
 * Autotuner of the fusion width: compiles the circuit for each candidate k
 * (0 = plain per-gate), applies it to q once untimed and once timed with HIP
 * events on q's stream, and leaves the circuit compiled with the fastest k.
 * q's state is overwritten by these runs.  The choice is cached per (qubit
 * count, precision, circuit contents) for the process, and appended to the
 * file named by QS_TUNE_CACHE when that variable is set (and read from it
 * first).  ms_out (may be NULL) receives num_candidates timings in ms.
 */
int qs_circuit_autotune(qs_qureg *q, qs_circuit *c, const int *candidates, int num_candidates, int *best_k,
                        double *ms_out);
/*
 * The same, and with try_specialized != 0 each candidate that compiles into
 * tile steps is timed a second time with its steps specialised
 * (qs_circuit_specialize; candidates the run-time compiler cannot build are
 * timed generic only).  The circuit is left compiled, and specialised if
 * that was faster, as the fastest of all timings says: *best_k receives the
 * width and *best_specialized (may be NULL) 1 for specialised steps.
 * ms_specialized_out (may be NULL) receives num_candidates timings in ms, -1
 * where no specialised form was timed.  Choices are cached as for
 * qs_circuit_autotune, separately for try_specialized = 0 and != 0.
 */
int qs_circuit_autotune_ex(qs_qureg *q, qs_circuit *c, const int *candidates, int num_candidates,
                           int try_specialized, int *best_k, int *best_specialized, double *ms_out,
                           double *ms_specialized_out);

/* ---- adjoint gradients of a statevector circuit --------------------------------- */

/*
 * Parametrised Pauli gadget exp(i * scale * params[param] * P) (Sec. "Pauli
 * gadget"; P a Pauli string on distinct qubits, codes 0..3) appended to a
 * statevector circuit; its angle is set by qs_circuit_set_params (0 until
 * then).  Density circuits: QS_E_PRECOND.
 */
int qs_circuit_add_param_gadget(qs_circuit *c, const int *targs, const int *paulis, int num_targs, int param,
                                double scale);
/* Sets every parametrised gadget's angle to scale * params[param].  The
 * circuit must be compiled again before qs_apply_circuit. */
int qs_circuit_set_params(qs_circuit *c, const double *params, int num_params);
/*
 * Energy E = <psi|H|psi> of H = sum_n coeffs[n] P_n (paulis: num_terms
 * strings of N codes, term-major) after the circuit, and dE/dparams[p] for
 * every parameter, by the adjoint method: psi (holding the initial state)
 * is run through the circuit one operator per pass, lambda = H psi (lam: a
 * statevector qureg of the same size, precision and stream, overwritten),
 * then for each operator from last to first dE/dtheta_p += -2 scale
 * Im <lambda|P|psi> for a parametrised gadget and psi, lambda <-
 * U^dag psi, U^dag lambda.  On return psi holds the initial state again (up
 * to rounding).  grads receives num_params values; energy one.  Sums in FP64.
 */
int qs_circuit_adjoint_gradient(qs_circuit *c, qs_qureg *psi, qs_qureg *lam, const int *paulis,
                                const double *coeffs, int num_terms, int num_params, double *energy,
                                double *grads);

/* ---- batches: many parametrised circuits of uneven size, with energies and
 *      adjoint gradients ------------------------------------------------------ */

/*
 * A batch holds many statevector circuits (1 <= N <= 30 qubits each) built
 * from single-qubit rotations exp(i * scale * params[p] * P) (P = X, Y or Z,
 * the Pauli gadget of Sec. "Pauli gadget" on one qubit), fixed single-qubit
 * gates and CZ gates, each circuit with its own Pauli-sum observable H and
 * parameter vector.  qs_batch_run starts every circuit from |0..0>, applies
 * it, and returns E = <psi|H|psi> per circuit; with gradients it also runs
 * the adjoint sweep: lambda = H psi, then for each operator from last to
 * first, dE/dtheta_p += 2 Re(i scale <lambda|P|phi>) for a rotation, and
 * phi, lambda <- U^dagger phi, U^dagger lambda.
 *
 * Execution: compile partitions every circuit into steps, each a set of at
 * most T qubits (T = 12 for complex64, 11 for complex128; every qubit when
 * N <= T) plus the operators that act inside it or are diagonal; a step
 * gathers each 2^T-amplitude tile of the state into LDS, applies its
 * operators there and writes the tile back.  Step s of every circuit runs
 * in one kernel launch; the whole run is captured once into a HIP graph.
 * Parameters are row-concatenated per circuit in creation order, as are the
 * returned gradients.  The batch owns its device buffers; its stream is the
 * one given to qs_batch_compile.  Calls on one batch must not overlap.
 */
typedef struct qs_batch qs_batch;
int qs_batch_create(int precision, qs_batch **out);
int qs_batch_destroy(qs_batch *b);
/* Adds a circuit of num_qubits qubits with num_params parameters; *index
 * receives its position. */
int qs_batch_add_circuit(qs_batch *b, int num_qubits, int num_params, int *index);
/* exp(i * scale * params[param] * P) on `qubit`, pauli 1 = X, 2 = Y, 3 = Z.
 * RY(a) = exp(-i a Y / 2) is pauli 2 with scale -0.5. */
int qs_batch_add_rotation(qs_batch *b, int circuit, int qubit, int pauli, int param, double scale);
/* The Pauli gadget exp(i * scale * params[param] * P) (Sec. "Pauli gadget")
 * of a Pauli string on num_targs distinct qubits (codes 0..3; identities
 * ignored, at least one non-identity), or with param = -1 the fixed gadget
 * exp(i * scale * P).  It is recorded as the rotation exp(i theta X) on one of
 * its qubits between parameter-free Clifford gates (basis changes and CZs
 * that map that rotation onto the gadget), so the adjoint sweep's gradient
 * with respect to the parameter is the gadget's.  Counts as one operator in
 * qs_batch_stats. */
int qs_batch_add_gadget(qs_batch *b, int circuit, const int *targs, const int *paulis, int num_targs,
                        int param, double scale);
/* A fixed 2 x 2 gate (row-major (re, im) doubles) on `qubit`. */
int qs_batch_add_gate1(qs_batch *b, int circuit, int qubit, const double *matrix);
/* Controlled-Z on two distinct qubits (diagonal, symmetric). */
int qs_batch_add_cz(qs_batch *b, int circuit, int q1, int q2);
/* Observable of a circuit: num_terms Pauli strings of N codes each (term-
 * major, qubit 0 first) with real coefficients. */
int qs_batch_set_observable(qs_batch *b, int circuit, const int *paulis, const double *coeffs, int num_terms);
/* Allocates the states (two per circuit), plans the steps, uploads the
 * tables and captures the graphs on hip_stream (NULL = null stream).
 * use_graph = 0 launches the kernels directly instead. */
int qs_batch_compile(qs_batch *b, void *hip_stream, int use_graph);
/* Runs the batch with the given parameters; energies receives one value per
 * circuit; grads (NULL to skip the adjoint sweep) one per parameter. */
int qs_batch_run(qs_batch *b, const double *params, double *energies, double *grads);
/* Copies circuit `circuit`'s statevector (2^N (re, im) doubles) as left by
 * the last run: the final state when that run skipped gradients. */
int qs_batch_get_state(qs_batch *b, int circuit, double *re_im);
/* Totals of the compiled batch; any pointer may be NULL.  logical_updates
 * counts 2^N per operator of every circuit (one forward application). */
int qs_batch_stats(const qs_batch *b, int *num_circuits, int *num_steps, uint64_t *total_amps,
                   uint64_t *logical_updates);
/* Specialises the compiled batch's register-path steps (tiles of at least
 * 2^9 amplitudes) at run time, as qs_circuit_specialize does for tile steps:
 * a step's phases and operators become compile-time constants of generated
 * kernels (one forward and one backward kernel per step index, switching
 * over the distinct step programs; circuits of the same structure share
 * theirs), compiled by $ROCM_PATH/llvm/bin/clang++ and loaded as modules;
 * the graphs are captured again.  Results equal those of the generic
 * kernels.  *num_programs (may be NULL) receives the number of distinct
 * programs.  QS_E_PRECOND if the batch is not compiled or has more than 512
 * programs (or 65536 operators in them): the generic kernels stay.  A
 * failed compilation (QS_E_HIP) also leaves the generic kernels.  Compiling
 * the batch again drops the specialisation. */
int qs_batch_specialize(qs_batch *b, int *num_programs);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_H */
