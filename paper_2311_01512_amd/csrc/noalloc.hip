// The Pauli-sum expectation value for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the same computation as qs_calc_expec_pauli_sum, on a caller's
// device buffer, with the reduction scratch in a file-scope device array.
#include "common.hpp"

#include <mutex>
#include <vector>

namespace qs {

// Reduction partials followed by the result slots: 256 KiB + 512 B, one copy
// per GPU the library runs on, held until the process ends.  On the host the
// name `scratch` only stands for the symbol; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address reaches kernels.  Every call on a GPU uses the same array
// and leaves its contents behind (each call's kernels write every partial
// and slot they later read), so calls that overlap on one GPU race.
constexpr size_t kScratchDoubles = kExpecPartials + kResultSlots;
static __device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_ptr;   // device address of `scratch`, by device ordinal

static int scratch_address(int dev, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(QS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" int qs_calc_expec_pauli_sum_noalloc(const void *amps, int num_qubits, int is_density, int precision,
                                               void *hip_stream, const int *paulis, const double *coeffs,
                                               int num_terms, double *out_re, double *out_im)
{
    if (!amps) return fail(QS_E_ARG, "null amplitudes");
    if (precision != QS_C64 && precision != QS_C128) return fail(QS_E_ARG, "bad precision");
    const int bits = is_density ? 2 * num_qubits : num_qubits;
    if (num_qubits < 1 || bits > 62) return fail(QS_E_ARG, "qubit count out of range");
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, amps) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QS_E_ARG, "amplitudes are not device memory known to HIP");
    }
    if (attr.type != hipMemoryTypeDevice || attr.device != dev)
        return fail(QS_E_ARG, "amplitudes must be device memory of the current device");
    double *dev_scratch = nullptr;
    int rc = scratch_address(dev, &dev_scratch);
    if (rc != QS_OK) return rc;
    // A qureg view of the caller's buffer whose scratch is the static array.
    // The partials and result slots that the reduction kernels need never
    // exceed it, whatever the state size or term count (kExpecPartials bounds
    // every launch); the view has no matrix staging ring (mat_ring_bytes = 0),
    // so no step can allocate one.
    double h_result[kResultSlots];
    qs_qureg q{};
    q.num_qubits = num_qubits;
    q.is_density = is_density ? 1 : 0;
    q.precision = precision;
    q.index_bits = bits;
    q.num_amps = 1ULL << bits;
    q.amps = const_cast<void *>(amps);
    q.owns_amps = 0;
    q.stream = (hipStream_t)hip_stream;
    q.device = dev;
    q.d_partials = dev_scratch;
    q.d_result = dev_scratch + kExpecPartials;
    q.h_result = h_result;
    q.mat_ring_bytes = 0;
    return expec_pauli_sum(&q, paulis, coeffs, num_terms, out_re, out_im);
}
