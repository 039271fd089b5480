// Qureg lifetime, initial states and host <-> device amplitude copies.
#include "common.hpp"

#include <cmath>

namespace qs {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

bool valid_qubits(const int *qs, int count, int n, std::string &why)
{
    if (count < 0) { why = "negative qubit count"; return false; }
    if (count > 0 && !qs) { why = "null qubit list"; return false; }
    for (int i = 0; i < count; i++) {
        if (qs[i] < 0 || qs[i] >= n) {
            why = "qubit " + std::to_string(qs[i]) + " outside [0, " + std::to_string(n) + ")";
            return false;
        }
        for (int j = 0; j < i; j++)
            if (qs[i] == qs[j]) {
                why = "qubit " + std::to_string(qs[i]) + " listed twice";
                return false;
            }
    }
    return true;
}

int stage_matrix(qs_qureg *q, const void *host, size_t bytes, const void **dev)
{
    const size_t aligned = (bytes + 255) & ~size_t(255);
    if (aligned > q->mat_ring_bytes) return fail(QS_E_ARG, "matrix larger than the staging ring");
    if (!q->d_mat_ring) {
        // allocated on the first matrix too large for kernel arguments
        if (hipMalloc(&q->d_mat_ring, q->mat_ring_bytes) != hipSuccess) {
            q->d_mat_ring = nullptr;
            (void)hipGetLastError();
            return fail(QS_E_ALLOC, "allocation of the matrix staging ring failed");
        }
        if (hipHostMalloc(&q->h_mat_ring, q->mat_ring_bytes, hipHostMallocDefault) != hipSuccess) {
            q->h_mat_ring = nullptr;
            (void)hipGetLastError();
            (void)hipFree(q->d_mat_ring);
            q->d_mat_ring = nullptr;
            return fail(QS_E_ALLOC, "allocation of the pinned matrix staging ring failed");
        }
        q->mat_ring_head = 0;
    }
    if (q->mat_ring_head + aligned > q->mat_ring_bytes) {
        // Wrapping: earlier copies out of the pinned ring must have finished.
        QS_HIP(hipStreamSynchronize(q->stream));
        q->mat_ring_head = 0;
    }
    unsigned char *h = q->h_mat_ring + q->mat_ring_head;
    unsigned char *d = q->d_mat_ring + q->mat_ring_head;
    std::memcpy(h, host, bytes);
    QS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, q->stream));
    q->mat_ring_head += aligned;
    *dev = d;
    return QS_OK;
}

// ---- initial-state kernels ---------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(256) void k_fill(C2<R> *__restrict__ a, uint64_t n, R re, R im,
                                               uint64_t one_index, int put_one)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        C2<R> v = mk<R>(re, im);
        if (put_one && i == one_index) v = mk<R>(R(1), R(0));
        a[i] = v;
    }
}

// SplitMix64 output number `counter` of a generator seeded with `seed`
// (Steele, Lea & Flood, OOPSLA 2014): state advanced counter+1 times by the
// golden-ratio increment, then the published finaliser.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

template <typename R>
__global__ __launch_bounds__(256) void k_hashed(C2<R> *__restrict__ a, uint64_t n, uint64_t seed, int exp_scale)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ur = 2.0 * ldexp((double)(splitmix64(seed, 2 * i) >> 11), -53) - 1.0;
        const double ui = 2.0 * ldexp((double)(splitmix64(seed, 2 * i + 1) >> 11), -53) - 1.0;
        a[i] = mk<R>((R)ldexp(ur, -exp_scale), (R)ldexp(ui, -exp_scale));
    }
}

// rho[j + k 2^N] = psi_j conj(psi_k)
template <typename R>
__global__ __launch_bounds__(256) void k_pure_density(C2<R> *__restrict__ rho, const C2<R> *__restrict__ psi, int N)
{
    const uint64_t n = 1ULL << (2 * N);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t mask = (1ULL << N) - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const C2<R> a = psi[i & mask], b = psi[i >> N];
        rho[i] = mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
    }
}

template <typename R>
static int launch_fill(qs_qureg *q, double re, double im, uint64_t one_index, int put_one)
{
    hipLaunchKernelGGL(k_fill<R>, dim3(grid_for(q->num_amps, 256)), dim3(256), 0, q->stream,
                       (C2<R> *)q->amps, q->num_amps, (R)re, (R)im, one_index, put_one);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

static int fill(qs_qureg *q, double re, double im, uint64_t one_index, int put_one)
{
    return q->precision == QS_C64 ? launch_fill<float>(q, re, im, one_index, put_one)
                                  : launch_fill<double>(q, re, im, one_index, put_one);
}

}  // namespace qs

using namespace qs;

#define QS_CHECK_Q(q)                                                    \
    do {                                                                 \
        if (!(q)) return fail(QS_E_ARG, "null qureg");                   \
    } while (0)

extern "C" {

const char *qs_last_error(void) { return g_last_error.c_str(); }

int qs_create_qureg(int num_qubits, int is_density, int precision, void *device_ptr, void *hip_stream,
                    qs_qureg **out)
{
    if (!out) return fail(QS_E_ARG, "null output pointer");
    *out = nullptr;
    if (precision != QS_C64 && precision != QS_C128) return fail(QS_E_ARG, "precision must be QS_C64 or QS_C128");
    if (num_qubits < 1) return fail(QS_E_ARG, "need at least one qubit");
    const int bits = is_density ? 2 * num_qubits : num_qubits;
    if (bits > 40) return fail(QS_E_ALLOC, "state of 2^" + std::to_string(bits) + " amplitudes is too large");
    const size_t amp_bytes = precision == QS_C64 ? 8 : 16;
    const uint64_t n = 1ULL << bits;

    qs_qureg *q = new (std::nothrow) qs_qureg{};
    if (!q) return fail(QS_E_ALLOC, "host allocation failed");
    q->num_qubits = num_qubits;
    q->is_density = is_density ? 1 : 0;
    q->precision = precision;
    q->index_bits = bits;
    q->num_amps = n;
    q->stream = (hipStream_t)hip_stream;
    q->mat_ring_bytes = kMatRingBytes;
    if (hipGetDevice(&q->device) != hipSuccess) {
        delete q;
        return fail(QS_E_HIP, "hipGetDevice failed");
    }
    auto cleanup = [&](int code, const std::string &msg) {
        qs_destroy_qureg(q);
        return fail(code, msg);
    };
    if (device_ptr) {
        q->amps = device_ptr;
        q->owns_amps = 0;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && n * amp_bytes > free_b)
            return cleanup(QS_E_ALLOC, "not enough free device memory for " + std::to_string(n * amp_bytes) + " bytes");
        if (hipMalloc(&q->amps, n * amp_bytes) != hipSuccess) {
            q->amps = nullptr;
            (void)hipGetLastError();
            return cleanup(QS_E_ALLOC, "hipMalloc of the amplitudes failed");
        }
        q->owns_amps = 1;
    }
    if (hipMalloc(&q->d_partials, sizeof(double) * 2 * kReduceBlocks * 4) != hipSuccess ||
        hipMalloc(&q->d_result, sizeof(double) * kResultSlots) != hipSuccess ||
        hipHostMalloc(&q->h_result, sizeof(double) * kResultSlots, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(QS_E_ALLOC, "scratch allocation failed");
    }
    *out = q;
    return QS_OK;
}

int qs_destroy_qureg(qs_qureg *q)
{
    if (!q) return QS_OK;
    if (q->stream || q->amps) (void)hipStreamSynchronize(q->stream);
    if (q->owns_amps && q->amps) (void)hipFree(q->amps);
    if (q->d_partials) (void)hipFree(q->d_partials);
    if (q->d_result) (void)hipFree(q->d_result);
    if (q->h_result) (void)hipHostFree(q->h_result);
    if (q->d_mat_ring) (void)hipFree(q->d_mat_ring);
    if (q->h_mat_ring) (void)hipHostFree(q->h_mat_ring);
    delete q;
    return QS_OK;
}

int qs_get_info(const qs_qureg *q, int *num_qubits, int *is_density, int *precision, uint64_t *num_amps,
                void **device_ptr)
{
    QS_CHECK_Q(q);
    if (num_qubits) *num_qubits = q->num_qubits;
    if (is_density) *is_density = q->is_density;
    if (precision) *precision = q->precision;
    if (num_amps) *num_amps = q->num_amps;
    if (device_ptr) *device_ptr = q->amps;
    return QS_OK;
}

int qs_set_stream(qs_qureg *q, void *hip_stream)
{
    QS_CHECK_Q(q);
    QS_HIP(hipStreamSynchronize(q->stream));
    q->stream = (hipStream_t)hip_stream;
    return QS_OK;
}

int qs_sync(qs_qureg *q)
{
    QS_CHECK_Q(q);
    QS_HIP(hipStreamSynchronize(q->stream));
    return QS_OK;
}

int qs_init_zero_state(qs_qureg *q)
{
    QS_CHECK_Q(q);
    return fill(q, 0.0, 0.0, 0, 1);
}

int qs_init_basis_state(qs_qureg *q, uint64_t index)
{
    QS_CHECK_Q(q);
    if (index >= (1ULL << q->num_qubits)) return fail(QS_E_ARG, "basis index out of range");
    const uint64_t i = q->is_density ? index * ((1ULL << q->num_qubits) + 1ULL) : index;
    return fill(q, 0.0, 0.0, i, 1);
}

int qs_init_plus_state(qs_qureg *q)
{
    QS_CHECK_Q(q);
    const double v = q->is_density ? std::ldexp(1.0, -q->num_qubits) : 1.0 / std::sqrt(std::ldexp(1.0, q->num_qubits));
    return fill(q, v, 0.0, 0, 0);
}

int qs_init_pure_density(qs_qureg *rho, const qs_qureg *psi)
{
    QS_CHECK_Q(rho);
    QS_CHECK_Q(psi);
    if (!rho->is_density || psi->is_density) return fail(QS_E_PRECOND, "need a density matrix and a statevector");
    if (rho->num_qubits != psi->num_qubits) return fail(QS_E_ARG, "qubit counts differ");
    if (rho->precision != psi->precision) return fail(QS_E_TYPE, "precisions differ");
    // psi's pending work must precede the read
    if (psi->stream != rho->stream) QS_HIP(hipStreamSynchronize(psi->stream));
    const unsigned grid = grid_for(rho->num_amps, 256);
    if (rho->precision == QS_C64)
        hipLaunchKernelGGL(k_pure_density<float>, dim3(grid), dim3(256), 0, rho->stream, (float2 *)rho->amps,
                           (const float2 *)psi->amps, rho->num_qubits);
    else
        hipLaunchKernelGGL(k_pure_density<double>, dim3(grid), dim3(256), 0, rho->stream, (double2 *)rho->amps,
                           (const double2 *)psi->amps, rho->num_qubits);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

int qs_init_hashed_state(qs_qureg *q, uint64_t seed)
{
    QS_CHECK_Q(q);
    const int e = (q->index_bits + 1) / 2;
    const unsigned grid = grid_for(q->num_amps, 256);
    if (q->precision == QS_C64)
        hipLaunchKernelGGL(k_hashed<float>, dim3(grid), dim3(256), 0, q->stream, (float2 *)q->amps, q->num_amps, seed, e);
    else
        hipLaunchKernelGGL(k_hashed<double>, dim3(grid), dim3(256), 0, q->stream, (double2 *)q->amps, q->num_amps, seed, e);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

int qs_set_amps(qs_qureg *q, uint64_t start, const double *re_im, uint64_t count)
{
    QS_CHECK_Q(q);
    if (count == 0) return QS_OK;
    if (!re_im) return fail(QS_E_ARG, "null host array");
    if (start > q->num_amps || count > q->num_amps - start) return fail(QS_E_ARG, "amplitude range out of bounds");
    QS_HIP(hipStreamSynchronize(q->stream));
    if (q->precision == QS_C128) {
        QS_HIP(hipMemcpy((double2 *)q->amps + start, re_im, count * 16, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(2 * count);
        for (uint64_t i = 0; i < 2 * count; i++) tmp[i] = (float)re_im[i];
        QS_HIP(hipMemcpy((float2 *)q->amps + start, tmp.data(), count * 8, hipMemcpyHostToDevice));
    }
    return QS_OK;
}

int qs_get_amps(const qs_qureg *q, uint64_t start, double *re_im, uint64_t count)
{
    QS_CHECK_Q(q);
    if (count == 0) return QS_OK;
    if (!re_im) return fail(QS_E_ARG, "null host array");
    if (start > q->num_amps || count > q->num_amps - start) return fail(QS_E_ARG, "amplitude range out of bounds");
    QS_HIP(hipStreamSynchronize(q->stream));
    if (q->precision == QS_C128) {
        QS_HIP(hipMemcpy(re_im, (const double2 *)q->amps + start, count * 16, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * count);
        QS_HIP(hipMemcpy(tmp.data(), (const float2 *)q->amps + start, count * 8, hipMemcpyDeviceToHost));
        for (uint64_t i = 0; i < 2 * count; i++) re_im[i] = tmp[i];
    }
    return QS_OK;
}

}  // extern "C"
