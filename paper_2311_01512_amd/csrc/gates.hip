// Amplitude-update kernels: the many-control many-target gate, the Pauli
// gadget, and their density-matrix forms (unitaries, superoperators, Kraus
// maps) on the Choi vector.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace qs {

using cd = std::complex<double>;

// Target bit masks of one launch, ascending: tb[p] = 1 << s[p].
struct TargBits {
    uint64_t b[6];
};

template <typename R, int NT> struct ArgMat {
    C2<R> m[(1 << NT) * (1 << NT)];
};

// Offset of local state l among a group's 2^NT amplitudes: bit p of l sets
// target bit tb[p].  l is a compile-time constant after unrolling, so this
// folds to scalar arithmetic.
template <int NT>
__device__ __forceinline__ uint64_t local_offset(const TargBits &tb, int l)
{
    uint64_t o = 0;
#pragma unroll
    for (int p = 0; p < NT; p++)
        if ((l >> p) & 1) o |= tb.b[p];
    return o;
}

// Many-control many-target gate (Eq. "local_manyqb_amp_update" under the
// control condition of Eq. "serial_manyctrl_ctrl_cond").  Thread-level unit
// = one group: the 2^NT amplitudes that differ only on the targets, located
// by splicing zeros at every control and target position into the group
// index and setting the control bits.  Matrix rows/columns are in ascending
// target order.  MAT_ARGS: matrix passed by value (NT <= 2), otherwise read
// from device memory into LDS once per block.
template <typename R, int NT, bool MAT_ARGS>
__global__ __launch_bounds__(256) void k_gate(C2<R> *__restrict__ a, uint64_t num_groups, InsertPlan plan,
                                               uint64_t ctrl_mask, TargBits tb, ArgMat<R, (MAT_ARGS ? NT : 1)> am,
                                               const C2<R> *__restrict__ gm)
{
    constexpr int D = 1 << NT;
    extern __shared__ unsigned char lds_raw[];
    C2<R> *lm = reinterpret_cast<C2<R> *>(lds_raw);
    if constexpr (!MAT_ARGS) {
        for (int i = threadIdx.x; i < D * D; i += blockDim.x) lm[i] = gm[i];
        __syncthreads();
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_groups; g += stride) {
        const uint64_t base = insert_zeros(g, plan) | ctrl_mask;
        C2<R> v[D];
#pragma unroll
        for (int l = 0; l < D; l++) v[l] = a[base | local_offset<NT>(tb, l)];
        if constexpr (MAT_ARGS) {
#pragma unroll
            for (int j = 0; j < D; j++) {
                C2<R> acc = mk<R>(R(0), R(0));
#pragma unroll
                for (int l = 0; l < D; l++) cmac<R>(acc, am.m[j * D + l], v[l]);
                a[base | local_offset<NT>(tb, j)] = acc;
            }
        } else {
            // Rows are not unrolled, so the LDS matrix reads stay inside the
            // loop instead of being hoisted into registers.
#pragma unroll 1
            for (int j = 0; j < D; j++) {
                C2<R> acc = mk<R>(R(0), R(0));
#pragma unroll
                for (int l = 0; l < D; l++) cmac<R>(acc, lm[j * D + l], v[l]);
                uint64_t o = 0;
#pragma unroll
                for (int p = 0; p < NT; p++)
                    if ((j >> p) & 1) o |= tb.b[p];
                a[base | o] = acc;
            }
        }
    }
}

// Pauli gadget exp(i theta P) (Sec. "Pauli gadget"): for the pair
// (i, j = i ^ xy) enumerated once, with c = i sin(theta) eta,
// Pairs are enumerated by splicing a zero at the HIGHEST flipped bit, so
// consecutive lanes touch consecutive amplitudes on both sides of the pair
// and every cache line is consumed by one wavefront (splicing at the lowest
// flipped bit would leave half of each line to a distant thread).
//   a_i <- cos(theta) a_i + c (-1)^{popc(j & yz)} a_j
//   a_j <- cos(theta) a_j + c (-1)^{popc(i & yz)} a_i.
template <typename R>
__global__ __launch_bounds__(256) void k_gadget_pairs(C2<R> *__restrict__ a, uint64_t num_pairs, uint64_t low_mask,
                                                       uint64_t xy, uint64_t yz, R cs, R c_re, R c_im)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_pairs; g += stride) {
        const uint64_t i = (g & low_mask) | ((g & ~low_mask) << 1);
        const uint64_t j = i ^ xy;
        const C2<R> ai = a[i], aj = a[j];
        const R si = (__popcll(i & yz) & 1) ? R(-1) : R(1);
        const R sj = (__popcll(j & yz) & 1) ? R(-1) : R(1);
        // c * s * x = s * (c_re x.x - c_im x.y, c_re x.y + c_im x.x)
        a[i] = mk<R>(fma(sj, c_re * aj.x - c_im * aj.y, cs * ai.x), fma(sj, c_re * aj.y + c_im * aj.x, cs * ai.y));
        a[j] = mk<R>(fma(si, c_re * ai.x - c_im * ai.y, cs * aj.x), fma(si, c_re * ai.y + c_im * ai.x, cs * aj.y));
    }
}

// Phase gadget (Eq. "phase_gadget_amp_change"): a_i <- e^{i theta s_i} a_i,
// s_i = (-1)^{popc(i & mask)}.
template <typename R>
__global__ __launch_bounds__(256) void k_gadget_diag(C2<R> *__restrict__ a, uint64_t n, uint64_t zmask, R cs, R sn)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const R s = (__popcll(i & zmask) & 1) ? -sn : sn;
        const C2<R> x = a[i];
        a[i] = mk<R>(cs * x.x - s * x.y, cs * x.y + s * x.x);
    }
}

// ---- host planning (step "launch plan": sort, permute, masks) --------------------------

// Reorders a 2^n x 2^n matrix whose index bit q belongs to targs[q] into one
// whose index bit p belongs to the p-th smallest target.
static std::vector<cd> permute_to_sorted(const std::vector<cd> &M, const std::vector<int> &targs,
                                         std::vector<int> &sorted_out)
{
    const int n = (int)targs.size();
    const int D = 1 << n;
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return targs[x] < targs[y]; });
    sorted_out.resize(n);
    for (int p = 0; p < n; p++) sorted_out[p] = targs[order[p]];
    std::vector<int> to_sorted(D);
    for (int j = 0; j < D; j++) {
        int s = 0;
        for (int p = 0; p < n; p++) s |= ((j >> order[p]) & 1) << p;
        to_sorted[j] = s;
    }
    std::vector<cd> out((size_t)D * D);
    for (int j = 0; j < D; j++)
        for (int l = 0; l < D; l++) out[(size_t)to_sorted[j] * D + to_sorted[l]] = M[(size_t)j * D + l];
    return out;
}

template <typename R, int NT>
static int launch_gate_t(qs_qureg *q, uint64_t num_groups, const InsertPlan &plan, uint64_t ctrl_mask,
                         const TargBits &tb, const std::vector<cd> &M)
{
    constexpr int D = 1 << NT;
    const unsigned grid = grid_for(num_groups, 256);
    if constexpr (NT <= 2) {
        ArgMat<R, NT> am;
        for (int i = 0; i < D * D; i++) am.m[i] = C2<R>{(R)M[i].real(), (R)M[i].imag()};
        hipLaunchKernelGGL((k_gate<R, NT, true>), dim3(grid), dim3(256), 0, q->stream, (C2<R> *)q->amps,
                           num_groups, plan, ctrl_mask, tb, am, (const C2<R> *)nullptr);
    } else {
        std::vector<C2<R>> hm(D * D);
        for (int i = 0; i < D * D; i++) hm[i] = C2<R>{(R)M[i].real(), (R)M[i].imag()};
        const void *dm = nullptr;
        int rc = stage_matrix(q, hm.data(), hm.size() * sizeof(C2<R>), &dm);
        if (rc != QS_OK) return rc;
        ArgMat<R, 1> dummy{};
        hipLaunchKernelGGL((k_gate<R, NT, false>), dim3(grid), dim3(256), D * D * sizeof(C2<R>), q->stream,
                           (C2<R> *)q->amps, num_groups, plan, ctrl_mask, tb, dummy, (const C2<R> *)dm);
    }
    QS_LAUNCH_CHECK();
    return QS_OK;
}

template <typename R>
static int launch_gate_r(qs_qureg *q, int nt, uint64_t num_groups, const InsertPlan &plan, uint64_t ctrl_mask,
                         const TargBits &tb, const std::vector<cd> &M)
{
    switch (nt) {
    case 1: return launch_gate_t<R, 1>(q, num_groups, plan, ctrl_mask, tb, M);
    case 2: return launch_gate_t<R, 2>(q, num_groups, plan, ctrl_mask, tb, M);
    case 3: return launch_gate_t<R, 3>(q, num_groups, plan, ctrl_mask, tb, M);
    case 4: return launch_gate_t<R, 4>(q, num_groups, plan, ctrl_mask, tb, M);
    case 5: return launch_gate_t<R, 5>(q, num_groups, plan, ctrl_mask, tb, M);
    case 6: return launch_gate_t<R, 6>(q, num_groups, plan, ctrl_mask, tb, M);
    default: return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    }
}

// Gate on the raw amplitude array viewed as index_bits qubits (a statevector,
// or a Choi vector treated as a 2N-qubit statevector).
int apply_raw_gate(qs_qureg *q, const std::vector<int> &ctrls, const std::vector<int> &targs,
                   const std::vector<cd> &M)
{
    const int nt = (int)targs.size(), nc = (int)ctrls.size();
    if (nt < 1 || nt > 6) return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    if (nc + nt > q->index_bits) return fail(QS_E_ARG, "more controls and targets than qubits");
    if (nc + nt > kMaxInsert) return fail(QS_E_ARG, "too many controls");
    std::vector<int> sorted;
    std::vector<cd> Ms = permute_to_sorted(M, targs, sorted);
    std::vector<int> all(ctrls);
    all.insert(all.end(), targs.begin(), targs.end());
    InsertPlan plan = make_insert_plan(all);
    uint64_t ctrl_mask = 0;
    for (int c : ctrls) ctrl_mask |= 1ULL << c;
    TargBits tb{};
    for (int p = 0; p < nt; p++) tb.b[p] = 1ULL << sorted[p];
    const uint64_t num_groups = 1ULL << (q->index_bits - nc - nt);
    return q->precision == QS_C64 ? launch_gate_r<float>(q, nt, num_groups, plan, ctrl_mask, tb, Ms)
                                  : launch_gate_r<double>(q, nt, num_groups, plan, ctrl_mask, tb, Ms);
}

// Pauli gadget on the raw array (index_bits qubits).
int apply_raw_gadget(qs_qureg *q, const std::vector<int> &targs, const std::vector<int> &paulis, double theta)
{
    uint64_t xy = 0, yz = 0;
    int ny = 0;
    for (size_t k = 0; k < targs.size(); k++) {
        const uint64_t b = 1ULL << targs[k];
        switch (paulis[k]) {
        case 0: break;
        case 1: xy |= b; break;
        case 2: xy |= b; yz |= b; ny++; break;
        case 3: yz |= b; break;
        default: return fail(QS_E_ARG, "Pauli codes are 0..3");
        }
    }
    const double cs = std::cos(theta), sn = std::sin(theta);
    const unsigned block = 256;
    if (xy == 0) {
        const uint64_t n = q->num_amps;
        if (q->precision == QS_C64)
            hipLaunchKernelGGL(k_gadget_diag<float>, dim3(grid_for(n, block)), dim3(block), 0, q->stream,
                               (float2 *)q->amps, n, yz, (float)cs, (float)sn);
        else
            hipLaunchKernelGGL(k_gadget_diag<double>, dim3(grid_for(n, block)), dim3(block), 0, q->stream,
                               (double2 *)q->amps, n, yz, cs, sn);
    } else {
        // c = i sin(theta) eta, eta = i^{#Y}
        const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
        const cd c = cd(0, sn) * eta[ny & 3];
        const int hb = 63 - __builtin_clzll(xy);
        const uint64_t low = (1ULL << hb) - 1ULL;
        const uint64_t np = q->num_amps >> 1;
        if (q->precision == QS_C64)
            hipLaunchKernelGGL(k_gadget_pairs<float>, dim3(grid_for(np, block)), dim3(block), 0, q->stream,
                               (float2 *)q->amps, np, low, xy, yz, (float)cs, (float)c.real(), (float)c.imag());
        else
            hipLaunchKernelGGL(k_gadget_pairs<double>, dim3(grid_for(np, block)), dim3(block), 0, q->stream,
                               (double2 *)q->amps, np, low, xy, yz, cs, c.real(), c.imag());
    }
    QS_LAUNCH_CHECK();
    return QS_OK;
}

static std::vector<cd> read_matrix(const double *m, int D)
{
    std::vector<cd> M((size_t)D * D);
    for (size_t i = 0; i < (size_t)D * D; i++) M[i] = cd(m[2 * i], m[2 * i + 1]);
    return M;
}

// Superoperator of a Kraus map (Eq. "superop_from_kraus_map"): entry (r, c)
// with r = i 2^n + k, c = j 2^n + l is sum_m conj(K_m[i][j]) K_m[k][l];
// the high half of each index acts on the shifted (t + N) qubits.
std::vector<cd> superop_of_kraus(const std::vector<std::vector<cd>> &ks, int n)
{
    const int d = 1 << n, D = d * d;
    std::vector<cd> S((size_t)D * D, cd(0, 0));
    for (const auto &K : ks)
        for (int r = 0; r < D; r++)
            for (int c = 0; c < D; c++)
                S[(size_t)r * D + c] += std::conj(K[(size_t)(r / d) * d + c / d]) * K[(size_t)(r % d) * d + c % d];
    return S;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_apply_multi_ctrl_multi_targ_unitary(qs_qureg *q, const int *ctrls, int num_ctrls, const int *targs,
                                           int num_targs, const double *matrix)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (!matrix) return fail(QS_E_ARG, "null matrix");
    if (num_targs < 1 || num_targs > 6) return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    if (num_ctrls < 0) return fail(QS_E_ARG, "negative control count");
    std::string why;
    std::vector<int> all;
    for (int i = 0; i < num_ctrls; i++) all.push_back(ctrls ? ctrls[i] : -1);
    for (int i = 0; i < num_targs; i++) all.push_back(targs ? targs[i] : -1);
    if (!valid_qubits(all.data(), (int)all.size(), q->num_qubits, why)) return fail(QS_E_ARG, why);
    std::vector<int> c(all.begin(), all.begin() + num_ctrls), t(all.begin() + num_ctrls, all.end());
    const int D = 1 << num_targs;
    std::vector<cd> M = read_matrix(matrix, D);
    if (!q->is_density) return apply_raw_gate(q, c, t, M);

    const int N = q->num_qubits;
    const int k = num_ctrls + num_targs;
    if (k <= 2) {
        // One pass of conj(U') (x) U' on (q, q + N), U' the controlled gate as a
        // dense matrix on (targets..., controls...), controls in the high bits.
        const int Dk = 1 << k;
        std::vector<cd> U((size_t)Dk * Dk, cd(0, 0));
        for (int i = 0; i < Dk; i++) U[(size_t)i * Dk + i] = 1.0;
        const int hi = (Dk - 1) & ~(D - 1);   // all control bits set
        for (int r = 0; r < D; r++)
            for (int cc = 0; cc < D; cc++) U[(size_t)(hi | r) * Dk + (hi | cc)] = M[(size_t)r * D + cc];
        std::vector<int> qs2 = t;
        qs2.insert(qs2.end(), c.begin(), c.end());
        std::vector<int> targs2 = qs2;
        for (int x : qs2) targs2.push_back(x + N);
        return apply_raw_gate(q, {}, targs2, superop_of_kraus({U}, k));
    }
    int rc = apply_raw_gate(q, c, t, M);
    if (rc != QS_OK) return rc;
    std::vector<int> c2(c), t2(t);
    for (int &x : c2) x += N;
    for (int &x : t2) x += N;
    for (auto &x : M) x = std::conj(x);
    return apply_raw_gate(q, c2, t2, M);
}

int qs_apply_pauli_gadget(qs_qureg *q, const int *targs, const int *paulis, int num_targs, double theta)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (num_targs < 1 || !targs || !paulis) return fail(QS_E_ARG, "need at least one target");
    std::string why;
    if (!valid_qubits(targs, num_targs, q->num_qubits, why)) return fail(QS_E_ARG, why);
    std::vector<int> t(targs, targs + num_targs), p(paulis, paulis + num_targs);
    for (int x : p)
        if (x < 0 || x > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
    int rc = apply_raw_gadget(q, t, p, theta);
    if (rc != QS_OK || !q->is_density) return rc;
    // conj(exp(i theta P)) = exp(i (-1)^{m+1} theta P), m = #Y, on t + N
    double th = -theta;
    for (int x : p)
        if (x == 2) th = -th;
    for (int &x : t) x += q->num_qubits;
    return apply_raw_gadget(q, t, p, th);
}

int qs_apply_superop(qs_qureg *q, const int *targs, int num_targs, const double *superop)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (!q->is_density) return fail(QS_E_PRECOND, "superoperators act on density matrices");
    if (num_targs < 1 || num_targs > 3 || !targs || !superop) return fail(QS_E_ARG, "1 to 3 targets supported");
    std::string why;
    if (!valid_qubits(targs, num_targs, q->num_qubits, why)) return fail(QS_E_ARG, why);
    std::vector<int> t2(targs, targs + num_targs);
    for (int i = 0; i < num_targs; i++) t2.push_back(targs[i] + q->num_qubits);
    return apply_raw_gate(q, {}, t2, read_matrix(superop, 1 << (2 * num_targs)));
}

int qs_apply_kraus_map(qs_qureg *q, const int *targs, int num_targs, const double *kraus, int num_ops)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (!q->is_density) return fail(QS_E_PRECOND, "Kraus maps act on density matrices");
    if (num_targs < 1 || num_targs > 3 || !targs || !kraus) return fail(QS_E_ARG, "1 to 3 targets supported");
    if (num_ops < 1) return fail(QS_E_ARG, "need at least one Kraus operator");
    std::string why;
    if (!valid_qubits(targs, num_targs, q->num_qubits, why)) return fail(QS_E_ARG, why);
    const int d = 1 << num_targs;
    std::vector<std::vector<cd>> ks;
    for (int m = 0; m < num_ops; m++) ks.push_back(read_matrix(kraus + (size_t)2 * m * d * d, d));
    std::vector<int> t2(targs, targs + num_targs);
    for (int i = 0; i < num_targs; i++) t2.push_back(targs[i] + q->num_qubits);
    return apply_raw_gate(q, {}, t2, superop_of_kraus(ks, num_targs));
}

}  // extern "C"
