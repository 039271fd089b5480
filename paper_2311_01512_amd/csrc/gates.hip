// Amplitude-update kernels: the many-control many-target gate, the Pauli
// gadget, and their density-matrix forms (unitaries, superoperators, Kraus
// maps) on the Choi vector.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace qs {



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
std::vector<cd> permute_to_sorted(const std::vector<cd> &M, const std::vector<int> &targs,
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

// ---- FP32 MFMA dense gate (complex64 state) -------------------------------------------
//
// The k-target gate as a real GEMM.  With G = Gr + i Gi (D x D, D = 2^k) and
// a tile X of 16 groups (D x 16 complex), Y = G X is computed as
//   [Yr; Yi] = [[Gr, -Gi], [Gi, Gr]] [Xr; Xi]
// by v_mfma_f32_16x16x4f32: M = 2D output rows in 16-row blocks, K = 2D rows
// of [Xr; Xi] in 4-row steps, N = 16 groups.  Lane L holds group L % 16;
// for K-step s it holds row 4 s + L / 16 of [Xr; Xi] (the B operand), which
// is the real (s < D/4) or imaginary part of one amplitude it loaded, and it
// receives output rows 4 (L / 16) + i of each 16-row block (i = 0..3).  The
// packed A operands (the big real matrix in MFMA lane order) sit in LDS.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int K>
__global__ __launch_bounds__(256) void k_dense_mfma(float2 *__restrict__ a, uint64_t num_tiles, InsertPlan plan,
                                                     uint64_t ctrl_mask, TargBits tb,
                                                     const f32x4 *__restrict__ apack)
{
    constexpr int D = 1 << K;
    constexpr int KS = 2 * D / 4;    // K-steps
    constexpr int MB = 2 * D / 16;   // 16-row output blocks
    constexpr int NA = MB * KS / 4;  // float4 A-operand packs per lane
    extern __shared__ f32x4 lds_a[];
    for (int i = threadIdx.x; i < NA * 64; i += blockDim.x) lds_a[i] = apack[i];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, rq = lane >> 4;
    // input row 4 s + rq: target bits 0-1 from rq (per lane), bits >= 2 from s
    const uint64_t off_in = ((rq & 1) ? tb.b[0] : 0) | ((rq & 2) ? tb.b[1] : 0);
    // output row 16 m + 4 rq + i: target bits 2-3 from rq (per lane)
    const uint64_t off_out = ((rq & 1) ? tb.b[2] : 0) | ((rq & 2) ? tb.b[3] : 0);
    const uint64_t num_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);

    // input offsets of this lane's D/4 amplitudes within a group
    uint64_t in_off[D / 4];
#pragma unroll
    for (int s = 0; s < D / 4; s++) {
        uint64_t o = off_in;
#pragma unroll
        for (int p = 2; p < K; p++)
            if ((s >> (p - 2)) & 1) o |= tb.b[p];
        in_off[s] = o;
    }
    uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= num_tiles) return;
    // software pipeline: the next tile's amplitudes are loaded while this
    // tile's MFMAs run (a wave walks tiles tile + k num_waves); the first
    // tile is waited for before the loop, so the loop never waits on stores
    float2 x[D / 4];
    {
        const uint64_t b0 = insert_zeros(tile * 16 + col, plan) | ctrl_mask;
#pragma unroll
        for (int s = 0; s < D / 4; s++) x[s] = a[b0 | in_off[s]];
#pragma unroll
        for (int s = 0; s < D / 4; s++) asm volatile("" ::"v"(x[s].x), "v"(x[s].y));
    }
    for (; tile < num_tiles; tile += num_waves) {
        // keep the LDS operand reads inside the loop (no hoisting into registers)
        asm volatile("" ::: "memory");
        const uint64_t base = insert_zeros(tile * 16 + col, plan) | ctrl_mask;
        const bool more = tile + num_waves < num_tiles;
        float2 nx[D / 4];
        if (more) {
            const uint64_t nb = insert_zeros((tile + num_waves) * 16 + col, plan) | ctrl_mask;
#pragma unroll
            for (int s = 0; s < D / 4; s++) nx[s] = a[nb | in_off[s]];
        }
        f32x4 acc[MB];
#pragma unroll
        for (int m = 0; m < MB; m++) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kq = 0; kq < KS / 4; kq++) {
#pragma unroll
            for (int m = 0; m < MB; m++) {
                const f32x4 av = lds_a[(m * (KS / 4) + kq) * 64 + lane];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int ks = 4 * kq + r;
                    const float bv = ks < D / 4 ? x[ks].x : x[ks - D / 4].y;
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv, acc[m], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < D / 16; m++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                uint64_t o = off_out | ((i & 1) ? tb.b[0] : 0) | ((i & 2) ? tb.b[1] : 0);
#pragma unroll
                for (int p = 4; p < K; p++)
                    if ((m >> (p - 4)) & 1) o |= tb.b[p];
                a[base | o] = make_float2(acc[m][i], acc[m + D / 16][i]);
            }
        }
        if (more) {
#pragma unroll
            for (int s = 0; s < D / 4; s++) x[s] = nx[s];
        }
    }
}

// Packs a D x D complex matrix (sorted target order) into the A-operand
// order of k_dense_mfma: element r of float4 number (m * KS/4 + kq) * 64 + L
// is B[16 m + L % 16][4 (4 kq + r) + L / 16] of the real matrix
// B = [[Gr, -Gi], [Gi, Gr]].
static void pack_mfma(const std::vector<cd> &Ms, int k, float *out)
{
    const int D = 1 << k, KS = 2 * D / 4, MB = 2 * D / 16;
    auto big = [&](int row, int c) -> double {
        const cd g = Ms[(size_t)(row % D) * D + (c % D)];
        const bool rim = row >= D, cim = c >= D;
        if (!rim && !cim) return g.real();
        if (!rim && cim) return -g.imag();
        if (rim && !cim) return g.imag();
        return g.real();
    };
    for (int m = 0; m < MB; m++)
        for (int kq = 0; kq < KS / 4; kq++)
            for (int L = 0; L < 64; L++)
                for (int r = 0; r < 4; r++)
                    out[(((size_t)m * (KS / 4) + kq) * 64 + L) * 4 + r] =
                        (float)big(16 * m + (L % 16), 4 * (4 * kq + r) + L / 16);
}

// ---- dense-gate launch interface ------------------------------------------------------------

size_t dense_matrix_bytes(int precision, int nt, int kernel)
{
    const size_t D = (size_t)1 << nt;
    if (kernel == kDenseMfma) return 4 * D * D * sizeof(float);
    if (nt <= 2) return 0;                               // passed by value
    return D * D * (precision == QS_C64 ? sizeof(float2) : sizeof(double2));
}

void pack_dense(int precision, int nt, int kernel, const std::vector<cd> &Ms, void *out)
{
    const size_t D = (size_t)1 << nt;
    if (kernel == kDenseMfma) {
        pack_mfma(Ms, nt, (float *)out);
    } else if (precision == QS_C64) {
        float2 *o = (float2 *)out;
        for (size_t i = 0; i < D * D; i++) o[i] = make_float2((float)Ms[i].real(), (float)Ms[i].imag());
    } else {
        double2 *o = (double2 *)out;
        for (size_t i = 0; i < D * D; i++) o[i] = make_double2(Ms[i].real(), Ms[i].imag());
    }
}

int choose_dense_kernel(int precision, int nt)
{
    const int pref = mfma_preference();
    if (precision != QS_C64 || nt < 4 || nt > 6) return kDenseVector;
    if (pref == 0) return kDenseVector;
    return kDenseMfma;
}

template <typename R, int NT>
static int launch_vector(qs_qureg *q, uint64_t num_groups, const InsertPlan &plan, uint64_t ctrl_mask,
                         const TargBits &tb, const std::vector<cd> &Ms, const void *dev)
{
    constexpr int D = 1 << NT;
    const unsigned grid = grid_for(num_groups, 256);
    if constexpr (NT <= 2) {
        ArgMat<R, NT> am;
        for (int i = 0; i < D * D; i++) am.m[i] = C2<R>{(R)Ms[i].real(), (R)Ms[i].imag()};
        hipLaunchKernelGGL((k_gate<R, NT, true>), dim3(grid), dim3(256), 0, q->stream, (C2<R> *)q->amps,
                           num_groups, plan, ctrl_mask, tb, am, (const C2<R> *)nullptr);
    } else {
        if (!dev) {
            std::vector<C2<R>> hm(D * D);
            pack_dense(q->precision, NT, kDenseVector, Ms, hm.data());
            int rc = stage_matrix(q, hm.data(), hm.size() * sizeof(C2<R>), &dev);
            if (rc != QS_OK) return rc;
        }
        ArgMat<R, 1> dummy{};
        hipLaunchKernelGGL((k_gate<R, NT, false>), dim3(grid), dim3(256), D * D * sizeof(C2<R>), q->stream,
                           (C2<R> *)q->amps, num_groups, plan, ctrl_mask, tb, dummy, (const C2<R> *)dev);
    }
    QS_LAUNCH_CHECK();
    return QS_OK;
}

template <int K>
static int launch_mfma(qs_qureg *q, uint64_t num_groups, const InsertPlan &plan, uint64_t ctrl_mask,
                       const TargBits &tb, const std::vector<cd> &Ms, const void *dev)
{
    constexpr int D = 1 << K;
    const size_t bytes = 4 * (size_t)D * D * sizeof(float);
    if (!dev) {
        std::vector<float> hm(4 * D * D);
        pack_mfma(Ms, K, hm.data());
        int rc = stage_matrix(q, hm.data(), bytes, &dev);
        if (rc != QS_OK) return rc;
    }
    const uint64_t tiles = num_groups / 16;   // num_groups is a multiple of 16 (checked by the caller)
    const uint64_t waves_per_block = 4;
    uint64_t blocks = (tiles + waves_per_block - 1) / waves_per_block;
    uint64_t cap = mfma_block_cap(K);
    if (cap > 0xFFFFFFFFull / 256) cap = 0xFFFFFFFFull / 256;   // 32-bit dispatch size in work-items
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL((k_dense_mfma<K>), dim3((unsigned)blocks), dim3(256), bytes, q->stream, (float2 *)q->amps,
                       tiles, plan, ctrl_mask, tb, (const f32x4 *)dev);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

template <typename R>
static int launch_vector_r(qs_qureg *q, int nt, uint64_t num_groups, const InsertPlan &plan, uint64_t ctrl_mask,
                           const TargBits &tb, const std::vector<cd> &Ms, const void *dev)
{
    switch (nt) {
    case 1: return launch_vector<R, 1>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    case 2: return launch_vector<R, 2>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    case 3: return launch_vector<R, 3>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    case 4: return launch_vector<R, 4>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    case 5: return launch_vector<R, 5>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    case 6: return launch_vector<R, 6>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
    default: return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    }
}

int launch_dense(qs_qureg *q, const std::vector<int> &ctrls, const std::vector<int> &sorted_targs,
                 const std::vector<cd> &Ms, const void *dev, int kernel)
{
    const int nt = (int)sorted_targs.size(), nc = (int)ctrls.size();
    if (nt < 1 || nt > 6) return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    if (nc + nt > q->index_bits) return fail(QS_E_ARG, "more controls and targets than qubits");
    if (nc + nt > kMaxInsert) return fail(QS_E_ARG, "too many controls");
    std::vector<int> all(ctrls);
    all.insert(all.end(), sorted_targs.begin(), sorted_targs.end());
    InsertPlan plan = make_insert_plan(all);
    uint64_t ctrl_mask = 0;
    for (int c : ctrls) ctrl_mask |= 1ULL << c;
    TargBits tb{};
    for (int p = 0; p < nt; p++) tb.b[p] = 1ULL << sorted_targs[p];
    const uint64_t num_groups = 1ULL << (q->index_bits - nc - nt);
    if (kernel == kDenseMfma && (q->precision != QS_C64 || nt < 4 || num_groups < 16)) {
        kernel = kDenseVector;
        dev = nullptr;   // a device copy in the MFMA layout does not fit the vector kernel
    }
    if (kernel == kDenseMfma) {
        switch (nt) {
        case 4: return launch_mfma<4>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
        case 5: return launch_mfma<5>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
        default: return launch_mfma<6>(q, num_groups, plan, ctrl_mask, tb, Ms, dev);
        }
    }
    return q->precision == QS_C64 ? launch_vector_r<float>(q, nt, num_groups, plan, ctrl_mask, tb, Ms, dev)
                                  : launch_vector_r<double>(q, nt, num_groups, plan, ctrl_mask, tb, Ms, dev);
}

// Gate on the raw amplitude array viewed as index_bits qubits (a statevector,
// or a Choi vector treated as a 2N-qubit statevector).
int apply_raw_gate(qs_qureg *q, const std::vector<int> &ctrls, const std::vector<int> &targs,
                   const std::vector<cd> &M)
{
    std::vector<int> sorted;
    std::vector<cd> Ms = permute_to_sorted(M, targs, sorted);
    const int nt = (int)targs.size();
    return launch_dense(q, ctrls, sorted, Ms, nullptr, choose_dense_kernel(q->precision, nt));
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
    if (q->is_density) return apply_density_gadget(q, targs, paulis, num_targs, theta);
    return apply_raw_gadget(q, t, p, theta);
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
