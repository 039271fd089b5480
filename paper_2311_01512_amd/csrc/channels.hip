// Bespoke decoherence channels on the Choi vector: one- and two-qubit
// dephasing, one- and two-qubit depolarising, amplitude damping.  Each is a
// single pass whose work unit is the group of amplitudes sharing every bit
// except the channel's "principal bits" (t and t + N for each target), with
// the closed-form update of the paper's channel sections instead of a dense
// superoperator: a dephasing pass leaves the amplitudes it does not change
// untouched (half of the state for one qubit, a quarter for two).
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace qs {

enum ChannelKind { kDephase1 = 0, kDephase2, kDepol1, kDepol2, kDamp };

// Principal bits of one launch: b[0] = t, b[1] = t + N (one qubit), or
// b[0] = t1, b[1] = t2, b[2] = t1 + N, b[3] = t2 + N (two qubits), as masks.
struct Principal {
    uint64_t b[4];
};

// Member m of a group (m < 4 or 16): bit p of m sets principal bit b[p].
template <int NB>
__device__ __forceinline__ uint64_t member(const Principal &pb, int m)
{
    uint64_t o = 0;
#pragma unroll
    for (int p = 0; p < NB; p++)
        if ((m >> p) & 1) o |= pb.b[p];
    return o;
}

template <typename R>
__device__ __forceinline__ C2<R> scale(C2<R> v, R f) { return mk<R>(f * v.x, f * v.y); }

// c0, c1, c2: the channel's coefficients, set on the host from p.
template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_channel(C2<R> *__restrict__ a, uint64_t num_groups, InsertPlan plan,
                                                  Principal pb, R c0, R c1, R c2)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < num_groups; g += stride) {
        const uint64_t base = insert_zeros(g, plan);
        if constexpr (KIND == kDephase1) {
            // Sec. "dephasing": i_t != i_{t+N} -> (1 - 2p) beta_i; c0 = 1 - 2p
            const uint64_t i1 = base | pb.b[0], i2 = base | pb.b[1];
            const C2<R> x1 = a[i1], x2 = a[i2];
            a[i1] = scale<R>(x1, c0);
            a[i2] = scale<R>(x2, c0);
        } else if constexpr (KIND == kDephase2) {
            // Eq. dephasing_2qb_update_rule: unless both principal pairs
            // agree, beta_i -> (1 - 4p/3) beta_i; c0 = 1 - 4p/3.  Member m:
            // bits 0, 1 = rows of t1, t2; bits 2, 3 = columns.
            C2<R> x[12];
            int k = 0;
#pragma unroll
            for (int m = 0; m < 16; m++) {
                if ((m & 3) == (m >> 2)) continue;
                x[k++] = a[base | member<4>(pb, m)];
            }
            k = 0;
#pragma unroll
            for (int m = 0; m < 16; m++) {
                if ((m & 3) == (m >> 2)) continue;
                a[base | member<4>(pb, m)] = scale<R>(x[k++], c0);
            }
        } else if constexpr (KIND == kDepol1) {
            // Eq. depolarising_1qb_amp_update: c0 = 1 - 2p/3, c1 = 2p/3,
            // c2 = 1 - 4p/3.  Member bit 0 = row bit t, bit 1 = column bit t+N.
            const uint64_t i00 = base, i10 = base | pb.b[0], i01 = base | pb.b[1], i11 = base | pb.b[0] | pb.b[1];
            const C2<R> x00 = a[i00], x10 = a[i10], x01 = a[i01], x11 = a[i11];
            a[i00] = mk<R>(c0 * x00.x + c1 * x11.x, c0 * x00.y + c1 * x11.y);
            a[i11] = mk<R>(c0 * x11.x + c1 * x00.x, c0 * x11.y + c1 * x00.y);
            a[i10] = scale<R>(x10, c2);
            a[i01] = scale<R>(x01, c2);
        } else if constexpr (KIND == kDepol2) {
            // Eq. 2qb_depolarising_choi_amp_update: the four members whose
            // principal pairs both agree (m = 0, 5, 10, 15) become
            // c0 beta_i + c1 (sum of the other three); every other member is
            // scaled by c2.  c0 = 1 - 4p/5, c1 = 4p/15, c2 = 1 - 16p/15.
            C2<R> x[16];
#pragma unroll
            for (int m = 0; m < 16; m++) x[m] = a[base | member<4>(pb, m)];
            const C2<R> s = mk<R>(x[0].x + x[5].x + x[10].x + x[15].x, x[0].y + x[5].y + x[10].y + x[15].y);
#pragma unroll
            for (int m = 0; m < 16; m++) {
                C2<R> y;
                if ((m & 3) == (m >> 2))
                    y = mk<R>(c0 * x[m].x + c1 * (s.x - x[m].x), c0 * x[m].y + c1 * (s.y - x[m].y));
                else
                    y = scale<R>(x[m], c2);
                a[base | member<4>(pb, m)] = y;
            }
        } else {
            // Eq. damping_amps_update: c0 = p, c1 = sqrt(1 - p), c2 = 1 - p.
            const uint64_t i00 = base, i10 = base | pb.b[0], i01 = base | pb.b[1], i11 = base | pb.b[0] | pb.b[1];
            const C2<R> x00 = a[i00], x10 = a[i10], x01 = a[i01], x11 = a[i11];
            a[i00] = mk<R>(x00.x + c0 * x11.x, x00.y + c0 * x11.y);
            a[i11] = scale<R>(x11, c2);
            a[i10] = scale<R>(x10, c1);
            a[i01] = scale<R>(x01, c1);
        }
    }
}

template <typename R>
static void launch_channel_r(qs_qureg *q, int kind, uint64_t groups, const InsertPlan &plan, const Principal &pb,
                             double c0, double c1, double c2)
{
    const int block = 256;
    const unsigned grid = grid_for(groups, block);
    C2<R> *amps = (C2<R> *)q->amps;
    switch (kind) {
    case kDephase1:
        hipLaunchKernelGGL((k_channel<R, kDephase1>), dim3(grid), dim3(block), 0, q->stream, amps, groups, plan, pb,
                           (R)c0, (R)c1, (R)c2);
        break;
    case kDephase2:
        hipLaunchKernelGGL((k_channel<R, kDephase2>), dim3(grid), dim3(block), 0, q->stream, amps, groups, plan, pb,
                           (R)c0, (R)c1, (R)c2);
        break;
    case kDepol1:
        hipLaunchKernelGGL((k_channel<R, kDepol1>), dim3(grid), dim3(block), 0, q->stream, amps, groups, plan, pb,
                           (R)c0, (R)c1, (R)c2);
        break;
    case kDepol2:
        hipLaunchKernelGGL((k_channel<R, kDepol2>), dim3(grid), dim3(block), 0, q->stream, amps, groups, plan, pb,
                           (R)c0, (R)c1, (R)c2);
        break;
    default:
        hipLaunchKernelGGL((k_channel<R, kDamp>), dim3(grid), dim3(block), 0, q->stream, amps, groups, plan, pb,
                           (R)c0, (R)c1, (R)c2);
        break;
    }
}

// Validates and launches a channel on targets t (1 or 2 of them).
static int apply_channel(qs_qureg *q, int kind, const int *t, int nt, double p, double c0, double c1, double c2)
{
    if (!q) return fail(QS_E_ARG, "null qureg");
    if (!q->is_density) return fail(QS_E_PRECOND, "decoherence channels act on density matrices");
    if (!(p >= 0.0 && p <= 1.0)) return fail(QS_E_ARG, "probability outside [0, 1]");
    std::string why;
    if (!valid_qubits(t, nt, q->num_qubits, why)) return fail(QS_E_ARG, why);
    const int N = q->num_qubits;
    Principal pb{};
    std::vector<int> bits;
    if (nt == 1) {
        pb.b[0] = 1ULL << t[0];
        pb.b[1] = 1ULL << (t[0] + N);
        bits = {t[0], t[0] + N};
    } else {
        pb.b[0] = 1ULL << t[0];
        pb.b[1] = 1ULL << t[1];
        pb.b[2] = 1ULL << (t[0] + N);
        pb.b[3] = 1ULL << (t[1] + N);
        bits = {t[0], t[1], t[0] + N, t[1] + N};
    }
    const InsertPlan plan = make_insert_plan(bits);
    const uint64_t groups = q->num_amps >> bits.size();
    if (q->precision == QS_C64)
        launch_channel_r<float>(q, kind, groups, plan, pb, c0, c1, c2);
    else
        launch_channel_r<double>(q, kind, groups, plan, pb, c0, c1, c2);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_apply_dephasing(qs_qureg *q, int target, double p)
{
    return apply_channel(q, kDephase1, &target, 1, p, 1.0 - 2.0 * p, 0.0, 0.0);
}

int qs_apply_two_qubit_dephasing(qs_qureg *q, int target1, int target2, double p)
{
    const int t[2] = {target1, target2};
    return apply_channel(q, kDephase2, t, 2, p, 1.0 - 4.0 * p / 3.0, 0.0, 0.0);
}

int qs_apply_depolarising(qs_qureg *q, int target, double p)
{
    return apply_channel(q, kDepol1, &target, 1, p, 1.0 - 2.0 * p / 3.0, 2.0 * p / 3.0, 1.0 - 4.0 * p / 3.0);
}

int qs_apply_two_qubit_depolarising(qs_qureg *q, int target1, int target2, double p)
{
    const int t[2] = {target1, target2};
    return apply_channel(q, kDepol2, t, 2, p, 1.0 - 4.0 * p / 5.0, 4.0 * p / 15.0, 1.0 - 16.0 * p / 15.0);
}

int qs_apply_damping(qs_qureg *q, int target, double p)
{
    return apply_channel(q, kDamp, &target, 1, p, p, std::sqrt(1.0 - p), 1.0 - p);
}

}  // extern "C"
