// Adjoint-method gradients of a recorded statevector circuit: parametrised
// Pauli gadgets exp(i scale theta_p P) (Sec. "Pauli gadget") of any weight
// among fixed gates and gadgets, for the energy E = <psi|H|psi> of a
// Pauli-sum observable H.
//
// Forward: psi = U_L .. U_1 psi_0, one pass per operator.  Then
// lambda = H psi and E = Re <psi|lambda>.  Backward, for k = L .. 1: if U_k
// is a parametrised gadget, dE/dtheta_p += 2 Re(i scale <lambda|P|psi>) =
// -2 scale Im <lambda|P|psi> (psi is then the state after U_k, lambda the
// back-propagated H psi); then psi <- U_k^dag psi and lambda <- U_k^dag lambda.
#include "circuit.hpp"

#include <algorithm>
#include <cmath>

namespace qs {

constexpr int kSumTerms = 16;   // Pauli terms per launch of the observable kernel

struct PauliTerms {
    int count;
    uint64_t x[kSumTerms], yz[kSumTerms];
    double cre[kSumTerms], cim[kSumTerms];   // h_n i^{#Y}
};

// out_i (+)= sum_n c_n (-1)^{popc(j & yz_n)} in_j, j = i ^ x_n: the Pauli
// action of Eq. "pauli_tensor_amp_update" (the factor taken at the source
// index j), summed over the terms.
template <typename R>
__global__ __launch_bounds__(256) void k_apply_pauli_sum(C2<R> *__restrict__ out, const C2<R> *__restrict__ in,
                                                          uint64_t n, PauliTerms t, int accumulate)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double re = 0.0, im = 0.0;
        if (accumulate) {
            const C2<R> o = out[i];
            re = o.x;
            im = o.y;
        }
        // eight terms' gathers in flight before their sums (same order of
        // additions as one term at a time)
        constexpr int G = 8;
        for (int k0 = 0; k0 < t.count; k0 += G) {
            C2<R> vs[G];
#pragma unroll
            for (int u = 0; u < G; u++)
                if (k0 + u < t.count) vs[u] = in[i ^ t.x[k0 + u]];
#pragma unroll
            for (int u = 0; u < G; u++) {
                if (k0 + u >= t.count) break;
                const int k = k0 + u;
                const uint64_t j = i ^ t.x[k];
                const C2<R> v = vs[u];
                const double s = (__popcll(j & t.yz[k]) & 1) ? -1.0 : 1.0;
                const double cr = s * t.cre[k], ci = s * t.cim[k];
                re += cr * (double)v.x - ci * (double)v.y;
                im += cr * (double)v.y + ci * (double)v.x;
            }
        }
        out[i] = mk<R>((R)re, (R)im);
    }
}

// Per-block partial sums of <a|P|b> = sum_i conj(a_i) beta_j b_j, j = i ^ x,
// beta_j = (-1)^{popc(j & yz)} (the factor i^{#Y} is applied on the host).
template <typename R>
__global__ __launch_bounds__(256) void k_inner_pauli(const C2<R> *__restrict__ a, const C2<R> *__restrict__ b,
                                                      uint64_t n, uint64_t x, uint64_t yz, double *__restrict__ partials)
{
    __shared__ double s_re[4], s_im[4];
    double re = 0.0, im = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t j = i ^ x;
        const C2<R> u = a[i], v = b[j];
        const double s = (__popcll(j & yz) & 1) ? -1.0 : 1.0;
        // conj(u) v
        re += s * ((double)u.x * (double)v.x + (double)u.y * (double)v.y);
        im += s * ((double)u.x * (double)v.y - (double)u.y * (double)v.x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_re[wave] = re;
        s_im[wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ((s_re[0] + s_re[1]) + s_re[2]) + s_re[3];
        partials[2 * blockIdx.x + 1] = ((s_im[0] + s_im[1]) + s_im[2]) + s_im[3];
    }
}

static void pauli_masks(const int *codes, int N, uint64_t &x, uint64_t &yz, int &ny)
{
    x = yz = 0;
    ny = 0;
    for (int k = 0; k < N; k++) {
        const int c = codes[k];
        if (c == 1 || c == 2) x |= 1ULL << k;
        if (c == 2 || c == 3) yz |= 1ULL << k;
        if (c == 2) ny++;
    }
}

template <typename R>
static int apply_observable(qs_qureg *lam, const qs_qureg *psi, const int *codes, const double *coeffs, int T)
{
    const int N = psi->num_qubits;
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    const unsigned grid = grid_for(psi->num_amps, 256);
    // T = 0: one launch with no terms writes zeros
    for (int b = 0; b < T || b == 0; b += kSumTerms) {
        PauliTerms t{};
        t.count = std::min(kSumTerms, T - b);   // 0 when T = 0
        for (int k = 0; k < t.count; k++) {
            int ny;
            pauli_masks(codes + (size_t)(b + k) * N, N, t.x[k], t.yz[k], ny);
            const cd c = coeffs[b + k] * eta[ny & 3];
            t.cre[k] = c.real();
            t.cim[k] = c.imag();
        }
        hipLaunchKernelGGL(k_apply_pauli_sum<R>, dim3(grid), dim3(256), 0, lam->stream, (C2<R> *)lam->amps,
                           (const C2<R> *)psi->amps, psi->num_amps, t, b > 0 ? 1 : 0);
        QS_LAUNCH_CHECK();
    }
    return QS_OK;
}

// <a|P|b> for the gadget string (targs, paulis), into out (re, im).
template <typename R>
static int inner_pauli(qs_qureg *a, const qs_qureg *b, const std::vector<int> &targs, const std::vector<int> &paulis,
                       double *out)
{
    uint64_t x = 0, yz = 0;
    int ny = 0;
    for (size_t k = 0; k < targs.size(); k++) {
        const uint64_t m = 1ULL << targs[k];
        if (paulis[k] == 1 || paulis[k] == 2) x |= m;
        if (paulis[k] == 2 || paulis[k] == 3) yz |= m;
        if (paulis[k] == 2) ny++;
    }
    const int blocks = (int)grid_for(a->num_amps, 256, kReduceBlocks);
    hipLaunchKernelGGL(k_inner_pauli<R>, dim3(blocks), dim3(256), 0, a->stream, (const C2<R> *)a->amps,
                       (const C2<R> *)b->amps, a->num_amps, x, yz, a->d_partials);
    QS_LAUNCH_CHECK();
    double v[2];
    int rc = finish_reduction(a, blocks, 0, v);
    if (rc != QS_OK) return rc;
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    const cd z = cd(v[0], v[1]) * eta[ny & 3];
    out[0] = z.real();
    out[1] = z.imag();
    return QS_OK;
}

static std::vector<cd> adjoint_of(const std::vector<cd> &M, size_t d)
{
    std::vector<cd> A(d * d);
    for (size_t r = 0; r < d; r++)
        for (size_t c = 0; c < d; c++) A[c * d + r] = std::conj(M[r * d + c]);
    return A;
}

static int apply_op(qs_qureg *q, const CircOp &op, bool adjoint)
{
    if (op.gadget) return apply_raw_gadget(q, op.targs, op.paulis, adjoint ? -op.theta : op.theta);
    if (!adjoint) return apply_raw_gate(q, op.ctrls, op.targs, op.M);
    return apply_raw_gate(q, op.ctrls, op.targs, adjoint_of(op.M, (size_t)1 << op.targs.size()));
}

template <typename R>
static int adjoint_sweep(const qs_circuit *c, qs_qureg *psi, qs_qureg *lam, const int *codes, const double *coeffs,
                         int T, int num_params, double *energy, double *grads)
{
    for (int p = 0; p < num_params; p++) grads[p] = 0.0;
    for (const auto &op : c->ops) {
        int rc = apply_op(psi, op, false);
        if (rc != QS_OK) return rc;
    }
    int rc = apply_observable<R>(lam, psi, codes, coeffs, T);
    if (rc != QS_OK) return rc;
    double re = 0.0, im = 0.0;
    rc = qs_calc_inner_product(psi, lam, &re, &im);
    if (rc != QS_OK) return rc;
    *energy = re;
    for (size_t k = c->ops.size(); k-- > 0;) {
        const CircOp &op = c->ops[k];
        if (op.gadget && op.param >= 0) {
            double z[2];
            rc = inner_pauli<R>(lam, psi, op.targs, op.paulis, z);
            if (rc != QS_OK) return rc;
            grads[op.param] += -2.0 * op.scale * z[1];
        }
        rc = apply_op(psi, op, true);
        if (rc == QS_OK) rc = apply_op(lam, op, true);
        if (rc != QS_OK) return rc;
    }
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_circuit_add_param_gadget(qs_circuit *c, const int *targs, const int *paulis, int num_targs, int param,
                                double scale)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (c->is_density) return fail(QS_E_PRECOND, "parametrised gadgets belong to statevector circuits");
    if (param < 0) return fail(QS_E_ARG, "negative parameter index");
    int rc = qs_circuit_add_pauli_gadget(c, targs, paulis, num_targs, 0.0);
    if (rc != QS_OK) return rc;
    c->ops.back().param = param;
    c->ops.back().scale = scale;
    return QS_OK;
}

int qs_circuit_set_params(qs_circuit *c, const double *params, int num_params)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (num_params < 0 || (num_params > 0 && !params)) return fail(QS_E_ARG, "bad parameter vector");
    for (const auto &op : c->ops)
        if (op.param >= num_params) return fail(QS_E_ARG, "parameter index beyond the vector");
    for (auto &op : c->ops)
        if (op.param >= 0) op.theta = op.scale * params[op.param];
    // compiled passes hold the old angles
    release_specialized(c);
    c->compiled = false;
    return QS_OK;
}

int qs_circuit_adjoint_gradient(qs_circuit *c, qs_qureg *psi, qs_qureg *lam, const int *paulis,
                                const double *coeffs, int num_terms, int num_params, double *energy, double *grads)
{
    if (!c || !psi || !lam || !energy || (num_params > 0 && !grads)) return fail(QS_E_ARG, "null argument");
    if (num_terms < 0 || (num_terms > 0 && (!paulis || !coeffs))) return fail(QS_E_ARG, "bad observable");
    if (c->is_density || psi->is_density || lam->is_density)
        return fail(QS_E_PRECOND, "adjoint gradients of statevector circuits");
    if (psi->num_qubits != c->num_qubits || lam->num_qubits != c->num_qubits)
        return fail(QS_E_ARG, "qubit counts differ");
    if (psi->precision != lam->precision) return fail(QS_E_TYPE, "precisions differ");
    if (psi->amps == lam->amps) return fail(QS_E_ARG, "psi and lambda must not alias");
    if (psi->stream != lam->stream) return fail(QS_E_ARG, "psi and lambda must share a stream");
    for (int i = 0; i < num_terms * c->num_qubits; i++)
        if (paulis[i] < 0 || paulis[i] > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
    for (const auto &op : c->ops)
        if (op.param >= num_params) return fail(QS_E_ARG, "parameter index beyond num_params");
    return psi->precision == QS_C64
               ? adjoint_sweep<float>(c, psi, lam, paulis, coeffs, num_terms, num_params, energy, grads)
               : adjoint_sweep<double>(c, psi, lam, paulis, coeffs, num_terms, num_params, energy, grads);
}

}  // extern "C"
