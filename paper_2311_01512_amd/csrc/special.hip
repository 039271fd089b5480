// The special unitaries of the paper's statevector sections, which need no
// dense matrix: SWAP gates (Sec. "Swap gate"), Pauli tensors (Sec. "Pauli
// tensor") and phase gadgets (Sec. "Phase gadget"), with their density-matrix
// forms from the conjugation identities of Alg.
// "distrib_dens_matr_specific_unitaries".  The paper applies those identities
// as two statevector passes over the Choi vector (targets t, then t + N); the
// operators on t and on t + N act on disjoint index bits and commute, so
// every density-matrix form here is one pass that reads and writes each
// amplitude at most once.  The Pauli gadget on a density matrix is fused the
// same way.
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace qs {

// ---- SWAP gates ----------------------------------------------------------------

// Disjoint SWAPs of up to kSwapPairs index-bit pairs per launch.  A group is
// the set of 4^P amplitudes that share every bit outside the P pairs; member
// m (its pair bits deposited at the pair positions) moves to the member with
// each pair's two bits exchanged.  The table lists every changed pair of
// members once, as offsets inside the group.
constexpr int kSwapPairs = 3;
constexpr int kSwapMoves = 28;   // (4^3 - 2^3) / 2

struct SwapTable {
    int num_moves;
    uint64_t from[kSwapMoves];
    uint64_t to[kSwapMoves];
};

// P pairs, NM = (4^P - 2^P) / 2 moves in batches of B: all loads of a batch
// are issued before its stores, so a thread keeps 2B loads in flight.  Every
// table index is a compile-time constant, so the table stays in kernel
// arguments.
template <typename R, int P>
__global__ __launch_bounds__(256) void k_swap(C2<R> *__restrict__ a, uint64_t num_groups, InsertPlan plan,
                                               SwapTable tab)
{
    constexpr int NM = ((1 << (2 * P)) - (1 << P)) / 2;
    constexpr int B = P == 3 ? 7 : NM;
    static_assert(NM % B == 0 && NM <= kSwapMoves, "swap batches");
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_groups; g += stride) {
        const uint64_t base = insert_zeros(g, plan);
#pragma clang loop unroll(full)
        for (int k0 = 0; k0 < NM; k0 += B) {
            R xr[B], xi[B], yr[B], yi[B];
#pragma clang loop unroll(full)
            for (int b = 0; b < B; b++) {
                const C2<R> u = a[base | tab.from[k0 + b]], v = a[base | tab.to[k0 + b]];
                xr[b] = u.x;
                xi[b] = u.y;
                yr[b] = v.x;
                yi[b] = v.y;
            }
#pragma clang loop unroll(full)
            for (int b = 0; b < B; b++) {
                a[base | tab.from[k0 + b]] = mk<R>(yr[b], yi[b]);
                a[base | tab.to[k0 + b]] = mk<R>(xr[b], xi[b]);
            }
        }
    }
}

// Swaps that involve one of the lowest index bits move amplitudes inside
// every 128-byte line, so each line is read and written whole whatever the
// kernel does.  Then a block stages one tile through LDS: the 2^T amplitudes
// that share every bit outside the tile bits (the pair bits and the lowest
// other bits), read in runs of consecutive amplitudes (16 bytes per lane),
// stored in LDS at their permuted local index, and written back in the same
// runs.
constexpr int kTileThreads = 256;

struct SwapTilePlan {
    InsertPlan outer;        // splices the T tile bits into the tile number
    uint64_t hi_bit[8];      // global mask of each tile-local bit above the lane bits
    int pairs;               // swapped local-bit pairs
    int ja[kSwapPairs], jb[kSwapPairs];
};

// Vectors of V = 16 bytes / amplitude size consecutive amplitudes; local bits
// 0..L-1 (L = log2(256 V)) are index bits 0..L-1 (lane and vector element),
// local bits L..T-1 are hi_bit[0..T-L-1].
template <typename R, int T>
__global__ __launch_bounds__(kTileThreads) void k_swap_tile(C2<R> *__restrict__ a, SwapTilePlan sp)
{
    constexpr int V = 16 / sizeof(C2<R>);
    constexpr int L = V == 2 ? 9 : 8;
    constexpr int E = (1 << T) / (kTileThreads * V);   // vectors per thread
    struct alignas(16) Vec {
        C2<R> v[V];
    };
    __shared__ Vec lds[(1 << T) / V];
    C2<R> *ldsa = &lds[0].v[0];
    const uint64_t base = insert_zeros(blockIdx.x, sp.outer) | ((uint64_t)threadIdx.x * V);
    Vec x[E];
#pragma unroll
    for (int k = 0; k < E; k++) {
        uint64_t off = 0;
#pragma unroll
        for (int b = 0; b < T - L; b++)
            if ((k >> b) & 1) off |= sp.hi_bit[b];
        x[k] = *(const Vec *)&a[base | off];
    }
#pragma unroll
    for (int k = 0; k < E; k++) {
#pragma unroll
        for (int e = 0; e < V; e++) {
            uint32_t m = (threadIdx.x * V + e) + (kTileThreads * V) * k;
            for (int p = 0; p < sp.pairs; p++) {
                const uint32_t d = ((m >> sp.ja[p]) ^ (m >> sp.jb[p])) & 1u;
                m ^= d * ((1u << sp.ja[p]) | (1u << sp.jb[p]));
            }
            ldsa[m] = x[k].v[e];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; k++) {
        uint64_t off = 0;
#pragma unroll
        for (int b = 0; b < T - L; b++)
            if ((k >> b) & 1) off |= sp.hi_bit[b];
        *(Vec *)&a[base | off] = lds[threadIdx.x + kTileThreads * k];
    }
}

// Tile bits of a staged swap: the pair bits and the lowest other bits, T in
// all, with the lane bits among them; false if the register is too small or
// the pairs leave too few low bits.
template <typename R, int T>
static bool launch_swap_tile(qs_qureg *q, const std::vector<int> &b1, const std::vector<int> &b2)
{
    constexpr int L = sizeof(C2<R>) == 8 ? 9 : 8;
    const int n = q->index_bits;
    if (n < T) return false;
    std::vector<char> in(n, 0);
    for (size_t k = 0; k < b1.size(); k++) in[b1[k]] = in[b2[k]] = 1;
    int need = T - 2 * (int)b1.size();
    for (int b = 0; b < n && need > 0; b++)
        if (!in[b]) {
            in[b] = 1;
            need--;
        }
    std::vector<int> tb;
    for (int b = 0; b < n; b++)
        if (in[b]) tb.push_back(b);
    if ((int)tb.size() != T || tb[L - 1] != L - 1) return false;
    SwapTilePlan sp{};
    sp.outer = make_insert_plan(tb);
    for (int k = 0; k < T - L; k++) sp.hi_bit[k] = 1ULL << tb[L + k];
    sp.pairs = (int)b1.size();
    for (int p = 0; p < sp.pairs; p++) {
        sp.ja[p] = (int)(std::find(tb.begin(), tb.end(), b1[p]) - tb.begin());
        sp.jb[p] = (int)(std::find(tb.begin(), tb.end(), b2[p]) - tb.begin());
    }
    const uint64_t tiles = q->num_amps >> T;
    hipLaunchKernelGGL((k_swap_tile<R, T>), dim3((unsigned)tiles), dim3(kTileThreads), 0, q->stream,
                       (C2<R> *)q->amps, sp);
    return true;
}

// Applies the disjoint index-bit swaps (lo[k], hi[k]) in launches of at most
// kSwapPairs pairs.
static int launch_swaps(qs_qureg *q, const std::vector<int> &b1, const std::vector<int> &b2)
{
    for (size_t p0 = 0; p0 < b1.size(); p0 += kSwapPairs) {
        const int P = (int)std::min<size_t>(kSwapPairs, b1.size() - p0);
        std::vector<int> bits;
        std::vector<uint64_t> m1(P), m2(P);
        for (int k = 0; k < P; k++) {
            bits.push_back(b1[p0 + k]);
            bits.push_back(b2[p0 + k]);
            m1[k] = 1ULL << b1[p0 + k];
            m2[k] = 1ULL << b2[p0 + k];
        }
        SwapTable tab{};
        for (int m = 0; m < (1 << (2 * P)); m++) {
            // member m: bit 2k sets pair k's first qubit, bit 2k+1 its second
            uint64_t off = 0, img = 0;
            int swapped = 0;
            for (int k = 0; k < P; k++) {
                const int u = (m >> (2 * k)) & 1, v = (m >> (2 * k + 1)) & 1;
                off |= (u ? m1[k] : 0) | (v ? m2[k] : 0);
                img |= (v ? m1[k] : 0) | (u ? m2[k] : 0);
                swapped |= (v + 2 * u) << (2 * k);
            }
            if (swapped > m) {   // each changed pair once
                tab.from[tab.num_moves] = off;
                tab.to[tab.num_moves] = img;
                tab.num_moves++;
            }
        }
        // a pair bit inside a 128-byte line (16 complex64 or 8 complex128
        // amplitudes): staged through LDS
        const int line_bits = q->precision == QS_C64 ? 4 : 3;
        if (*std::min_element(bits.begin(), bits.end()) < line_bits) {
            const std::vector<int> c1(b1.begin() + p0, b1.begin() + p0 + P), c2(b2.begin() + p0, b2.begin() + p0 + P);
            const bool staged = q->precision == QS_C64 ? launch_swap_tile<float, 12>(q, c1, c2)
                                                       : launch_swap_tile<double, 11>(q, c1, c2);
            if (staged) {
                QS_LAUNCH_CHECK();
                continue;
            }
        }
        const InsertPlan plan = make_insert_plan(bits);
        const uint64_t groups = q->num_amps >> (2 * P);
        const int block = 256;
        const unsigned grid = grid_for(groups, block);
        C2<float> *a32 = (C2<float> *)q->amps;
        C2<double> *a64 = (C2<double> *)q->amps;
        const bool f32 = q->precision == QS_C64;
        switch (P) {
        case 1:
            if (f32) hipLaunchKernelGGL((k_swap<float, 1>), dim3(grid), dim3(block), 0, q->stream, a32, groups, plan, tab);
            else hipLaunchKernelGGL((k_swap<double, 1>), dim3(grid), dim3(block), 0, q->stream, a64, groups, plan, tab);
            break;
        case 2:
            if (f32) hipLaunchKernelGGL((k_swap<float, 2>), dim3(grid), dim3(block), 0, q->stream, a32, groups, plan, tab);
            else hipLaunchKernelGGL((k_swap<double, 2>), dim3(grid), dim3(block), 0, q->stream, a64, groups, plan, tab);
            break;
        default:
            if (f32) hipLaunchKernelGGL((k_swap<float, 3>), dim3(grid), dim3(block), 0, q->stream, a32, groups, plan, tab);
            else hipLaunchKernelGGL((k_swap<double, 3>), dim3(grid), dim3(block), 0, q->stream, a64, groups, plan, tab);
            break;
        }
        QS_LAUNCH_CHECK();
    }
    return QS_OK;
}

// ---- Pauli tensors ---------------------------------------------------------------

// x times i^k.
template <typename R>
__device__ __forceinline__ C2<R> times_i_pow(C2<R> x, uint32_t k)
{
    const R re = (k & 1) ? -x.y : x.x;
    const R im = (k & 1) ? x.x : x.y;
    return (k & 2) ? mk<R>(-re, -im) : mk<R>(re, im);
}

// Pauli tensor (Eq. "pauli_tensor_amp_update"): for the pair
// (i, j = i ^ xy), enumerated once by splicing a zero in at the highest
// flipped bit, a_i <- beta_j a_j and a_j <- beta_i a_i, where
// beta_x = i^e (-1)^{popc(x & yz)} (e = number of Y, mod 4).  Only unit
// factors: no floating-point arithmetic beyond sign changes.
template <typename R>
__global__ __launch_bounds__(256) void k_pauli_pairs(C2<R> *__restrict__ a, uint64_t num_pairs, uint64_t low_mask,
                                                      uint64_t xy, uint64_t yz, uint32_t e)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_pairs; g += stride) {
        const uint64_t i = (g & low_mask) | ((g & ~low_mask) << 1);
        const uint64_t j = i ^ xy;
        const C2<R> ai = a[i], aj = a[j];
        a[i] = times_i_pow<R>(aj, e + 2u * (uint32_t)(__popcll(j & yz) & 1));
        a[j] = times_i_pow<R>(ai, e + 2u * (uint32_t)(__popcll(i & yz) & 1));
    }
}

// Pauli tensor of Z and identity only, times i^e: a sign per amplitude.
template <typename R>
__global__ __launch_bounds__(256) void k_pauli_diag(C2<R> *__restrict__ a, uint64_t n, uint64_t yz, uint32_t e)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        a[i] = times_i_pow<R>(a[i], e + 2u * (uint32_t)(__popcll(i & yz) & 1));
}

struct PauliMasks {
    uint64_t xy = 0, yz = 0;
    int ny = 0;
};

static bool pauli_masks_of(const int *targs, const int *paulis, int n, PauliMasks &pm)
{
    for (int k = 0; k < n; k++) {
        const uint64_t b = 1ULL << targs[k];
        switch (paulis[k]) {
        case 0: break;
        case 1: pm.xy |= b; break;
        case 2: pm.xy |= b; pm.yz |= b; pm.ny++; break;
        case 3: pm.yz |= b; break;
        default: return false;
        }
    }
    return true;
}

static int launch_pauli_tensor(qs_qureg *q, uint64_t xy, uint64_t yz, uint32_t e)
{
    const int block = 256;
    e &= 3u;
    if (xy == 0) {
        // the identity needs no pass
        if (yz == 0 && e == 0) return QS_OK;
        const uint64_t n = q->num_amps;
        if (q->precision == QS_C64)
            hipLaunchKernelGGL(k_pauli_diag<float>, dim3(grid_for(n, block)), dim3(block), 0, q->stream,
                               (float2 *)q->amps, n, yz, e);
        else
            hipLaunchKernelGGL(k_pauli_diag<double>, dim3(grid_for(n, block)), dim3(block), 0, q->stream,
                               (double2 *)q->amps, n, yz, e);
    } else {
        const int hb = 63 - __builtin_clzll(xy);
        const uint64_t low = (1ULL << hb) - 1ULL;
        const uint64_t np = q->num_amps >> 1;
        if (q->precision == QS_C64)
            hipLaunchKernelGGL(k_pauli_pairs<float>, dim3(grid_for(np, block)), dim3(block), 0, q->stream,
                               (float2 *)q->amps, np, low, xy, yz, e);
        else
            hipLaunchKernelGGL(k_pauli_pairs<double>, dim3(grid_for(np, block)), dim3(block), 0, q->stream,
                               (double2 *)q->amps, np, low, xy, yz, e);
    }
    QS_LAUNCH_CHECK();
    return QS_OK;
}

// ---- Pauli and phase gadgets on density matrices ----------------------------------

// exp(i th1 P) on targets t times exp(i th2 P') on t + N, P' = P shifted by N
// bits, in one pass.  Diagonal case (Z only): amplitude i is multiplied by
// ph[s1 + 2 s2], s1 = popc(i & zlo) & 1, s2 = popc(i & zhi) & 1, the four
// phases e^{i (+-th1 +- th2)} computed on the host.
template <typename R>
__global__ __launch_bounds__(256) void k_dm_phase(C2<R> *__restrict__ a, uint64_t n, uint64_t zlo, uint64_t zhi,
                                                   C2<R> p0, C2<R> p1, C2<R> p2, C2<R> p3)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int s1 = __popcll(i & zlo) & 1, s2 = __popcll(i & zhi) & 1;
        const C2<R> lo = s1 ? p1 : p0, hi = s1 ? p3 : p2;
        a[i] = cmul<R>(s2 ? hi : lo, a[i]);
    }
}

// Non-diagonal case.  With G1 = c1 + i s1 P on t and G2 = c2 + i s2 P' on
// t + N (Euler form of Sec. "Pauli gadget"), G2 G1 couples the four
// amplitudes i_u = i0 ^ (u&1 ? x1 : 0) ^ (u&2 ? x2 : 0):
//   a'_u = A a_u + B b1(u^1) a_{u^1} + C b2(u^2) a_{u^2} + D b1(u^1) b2(u^2) a_{u^3}
// with A = c1 c2, B = i s1 c2 eta, C = i c1 s2 eta, D = -s1 s2 eta^2,
// eta = i^{#Y}, and b1(v) = (-1)^{popc(i_v & yz1)}, b2(v) = (-1)^{popc(i_v &
// yz2)}.  (yz2 lies above bit N and x1 below it, so b2 of i_{u^3} equals b2
// of i_{u^2}.)  Groups are enumerated by splicing zeros in at the highest
// bits of x1 and x2.
template <typename R>
__global__ __launch_bounds__(256) void k_dm_gadget(C2<R> *__restrict__ a, uint64_t num_groups, InsertPlan plan,
                                                    uint64_t x1, uint64_t x2, uint64_t yz1, uint64_t yz2, R A,
                                                    C2<R> B, C2<R> C, C2<R> D)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_groups; g += stride) {
        const uint64_t i0 = insert_zeros(g, plan);
        uint64_t idx[4];
        C2<R> x[4];
        int b1[4], b2[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            idx[u] = i0 ^ ((u & 1) ? x1 : 0) ^ ((u & 2) ? x2 : 0);
            x[u] = a[idx[u]];
            b1[u] = __popcll(idx[u] & yz1) & 1;
            b2[u] = __popcll(idx[u] & yz2) & 1;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const C2<R> v1 = x[u ^ 1], v2 = x[u ^ 2], v3 = x[u ^ 3];
            const R f1 = b1[u ^ 1] ? R(-1) : R(1);
            const R f2 = b2[u ^ 2] ? R(-1) : R(1);
            const R f3 = f1 * f2;
            C2<R> acc = mk<R>(A * x[u].x, A * x[u].y);
            cmac<R>(acc, mk<R>(f1 * B.x, f1 * B.y), v1);
            cmac<R>(acc, mk<R>(f2 * C.x, f2 * C.y), v2);
            cmac<R>(acc, mk<R>(f3 * D.x, f3 * D.y), v3);
            a[idx[u]] = acc;
        }
    }
}

template <typename R>
static void launch_dm_phase_r(qs_qureg *q, uint64_t zlo, uint64_t zhi, const cd ph[4])
{
    const int block = 256;
    const uint64_t n = q->num_amps;
    C2<R> p[4];
    for (int k = 0; k < 4; k++) p[k] = C2<R>{(R)ph[k].real(), (R)ph[k].imag()};
    hipLaunchKernelGGL(k_dm_phase<R>, dim3(grid_for(n, block)), dim3(block), 0, q->stream, (C2<R> *)q->amps, n, zlo,
                       zhi, p[0], p[1], p[2], p[3]);
}

template <typename R>
static void launch_dm_gadget_r(qs_qureg *q, const InsertPlan &plan, uint64_t groups, const PauliMasks &lo,
                               const PauliMasks &hi, double A, cd B, cd C, cd D)
{
    const int block = 256;
    hipLaunchKernelGGL(k_dm_gadget<R>, dim3(grid_for(groups, block)), dim3(block), 0, q->stream, (C2<R> *)q->amps,
                       groups, plan, lo.xy, hi.xy, lo.yz, hi.yz, (R)A, C2<R>{(R)B.real(), (R)B.imag()},
                       C2<R>{(R)C.real(), (R)C.imag()}, C2<R>{(R)D.real(), (R)D.imag()});
}

// rho -> G rho G^dagger for the gadget G = exp(i theta P): exp(i theta P) on
// t and exp(i (-1)^{m+1} theta P) on t + N (m = number of Y), one pass.
static int apply_dm_gadget(qs_qureg *q, const PauliMasks &pm, double theta)
{
    const int N = q->num_qubits;
    PauliMasks hi;
    hi.xy = pm.xy << N;
    hi.yz = pm.yz << N;
    hi.ny = pm.ny;
    const double th1 = theta, th2 = (pm.ny & 1) ? theta : -theta;
    if (pm.xy == 0) {
        if (pm.yz == 0) {
            // P = identity: G = e^{i theta}, G rho G^dagger = rho
            return QS_OK;
        }
        // phases e^{i (th1 s1 + th2 s2)}, s = +1 for even parity
        cd ph[4];
        for (int k = 0; k < 4; k++) {
            const double s1 = (k & 1) ? -1.0 : 1.0, s2 = (k & 2) ? -1.0 : 1.0;
            ph[k] = std::polar(1.0, th1 * s1 + th2 * s2);
        }
        if (q->precision == QS_C64)
            launch_dm_phase_r<float>(q, pm.yz, hi.yz, ph);
        else
            launch_dm_phase_r<double>(q, pm.yz, hi.yz, ph);
        QS_LAUNCH_CHECK();
        return QS_OK;
    }
    const cd eta_tab[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    const cd eta = eta_tab[pm.ny & 3];
    const double c1 = std::cos(th1), s1 = std::sin(th1), c2 = std::cos(th2), s2 = std::sin(th2);
    const double A = c1 * c2;
    const cd B = cd(0, s1 * c2) * eta, C = cd(0, c1 * s2) * eta, D = -s1 * s2 * eta * eta;
    const int hb = 63 - __builtin_clzll(pm.xy);
    const InsertPlan plan = make_insert_plan({hb, hb + N});
    const uint64_t groups = q->num_amps >> 2;
    if (q->precision == QS_C64)
        launch_dm_gadget_r<float>(q, plan, groups, pm, hi, A, B, C, D);
    else
        launch_dm_gadget_r<double>(q, plan, groups, pm, hi, A, B, C, D);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

static int check_paulis(qs_qureg *q, const int *targs, const int *paulis, int n, PauliMasks &pm)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (n < 1 || !targs || !paulis) return fail(QS_E_ARG, "need at least one target");
    std::string why;
    if (!valid_qubits(targs, n, q->num_qubits, why)) return fail(QS_E_ARG, why);
    if (!pauli_masks_of(targs, paulis, n, pm)) return fail(QS_E_ARG, "Pauli codes are 0..3");
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_apply_swap(qs_qureg *q, int qubit1, int qubit2)
{
    return qs_apply_multi_swap(q, &qubit1, &qubit2, 1);
}

int qs_apply_multi_swap(qs_qureg *q, const int *qubits1, const int *qubits2, int num_pairs)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (num_pairs < 1 || !qubits1 || !qubits2) return fail(QS_E_ARG, "need at least one pair");
    const int N = q->num_qubits;
    if (2 * num_pairs > N) return fail(QS_E_ARG, "more swapped qubits than the register holds");
    std::vector<int> all(qubits1, qubits1 + num_pairs);
    all.insert(all.end(), qubits2, qubits2 + num_pairs);
    std::string why;
    if (!valid_qubits(all.data(), (int)all.size(), N, why)) return fail(QS_E_ARG, why);
    std::vector<int> b1(qubits1, qubits1 + num_pairs), b2(qubits2, qubits2 + num_pairs);
    if (q->is_density) {
        // conj(SWAP) = SWAP: the same swaps on the column bits t + N
        for (int k = 0; k < num_pairs; k++) {
            b1.push_back(qubits1[k] + N);
            b2.push_back(qubits2[k] + N);
        }
    }
    return launch_swaps(q, b1, b2);
}

int qs_apply_pauli_tensor(qs_qureg *q, const int *targs, const int *paulis, int num_targs)
{
    PauliMasks pm;
    const int rc = check_paulis(q, targs, paulis, num_targs, pm);
    if (rc != QS_OK) return rc;
    if (!q->is_density) return launch_pauli_tensor(q, pm.xy, pm.yz, (uint32_t)pm.ny);
    // P on t, P on t + N, then (-1)^m (conj(P) = (-1)^m P, m = number of Y):
    // one Pauli string on both halves whose factor is i^m i^m (-1)^m = 1
    const int N = q->num_qubits;
    const uint32_t e = (uint32_t)(pm.ny + pm.ny + 2 * pm.ny);
    return launch_pauli_tensor(q, pm.xy | (pm.xy << N), pm.yz | (pm.yz << N), e);
}

int qs_apply_phase_gadget(qs_qureg *q, const int *targs, int num_targs, double theta)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (num_targs < 1 || num_targs > 64 || !targs) return fail(QS_E_ARG, "need at least one target");
    std::vector<int> z((size_t)num_targs, 3);
    PauliMasks pm;
    const int rc = check_paulis(q, targs, z.data(), num_targs, pm);
    if (rc != QS_OK) return rc;
    if (q->is_density) return apply_dm_gadget(q, pm, theta);
    return apply_raw_gadget(q, std::vector<int>(targs, targs + num_targs), z, theta);
}

}  // extern "C"

namespace qs {

// Pauli gadget on a density matrix in one pass (used by qs_apply_pauli_gadget).
int apply_density_gadget(qs_qureg *q, const int *targs, const int *paulis, int num_targs, double theta)
{
    PauliMasks pm;
    const int rc = check_paulis(q, targs, paulis, num_targs, pm);
    if (rc != QS_OK) return rc;
    return apply_dm_gadget(q, pm, theta);
}

}  // namespace qs
