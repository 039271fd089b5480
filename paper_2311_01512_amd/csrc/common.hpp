// Shared definitions of the gfx950 simulator library: amplitude types,
// bit-index algebra, the qureg object and error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsim.h"
#include "dev_core.hpp"

namespace qs {

// Every entry point bounds the number of positions it splices before it gets
// here; a longer list yields an empty plan (n = -1, which inserts nothing)
// instead of writing past the fixed arrays.
inline InsertPlan make_insert_plan(std::vector<int> qubits)
{
    InsertPlan p{};
    if (qubits.size() > (size_t)kMaxInsert) {
        p.n = -1;
        return p;
    }
    std::vector<int> s = qubits;
    for (size_t i = 1; i < s.size(); i++)       // insertion sort, tiny lists
        for (size_t j = i; j > 0 && s[j - 1] > s[j]; j--) std::swap(s[j - 1], s[j]);
    p.n = (int)s.size();
    for (int k = 0; k < p.n; k++) p.low[k] = (1ULL << s[k]) - 1ULL;
    return p;
}

// ---- qureg ---------------------------------------------------------------------

}  // namespace qs

struct qs_qureg {
    int num_qubits;      // N
    int is_density;
    int precision;       // QS_C64 / QS_C128
    int index_bits;      // N, or 2N for a density matrix
    uint64_t num_amps;   // 2^index_bits
    void *amps;          // device amplitudes
    int owns_amps;
    hipStream_t stream;
    int device;
    // scratch owned by the qureg
    double *d_partials;  // per-block partial sums of reductions
    double *d_result;    // final reduction results
    double *h_result;    // pinned host copy of d_result
    unsigned char *d_mat_ring;  // device copies of large gate matrices
    unsigned char *h_mat_ring;  // pinned host staging of the same
    size_t mat_ring_bytes;
    size_t mat_ring_head;
};

namespace qs {

constexpr int kReduceBlocks = 16384;      // partial sums per reduction pass
constexpr int kResultSlots = 64;          // doubles in d_result / h_result
constexpr size_t kMatRingBytes = 4u << 20;

// ---- errors -------------------------------------------------------------------

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define QS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::qs::fail(QS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define QS_LAUNCH_CHECK()                                                              \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return ::qs::fail(QS_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

// Validates that qubits are distinct and inside [0, n).
bool valid_qubits(const int *qs, int count, int n, std::string &why);

// Launch geometry of the streaming kernels: one unit of work per thread (a
// grid of ceil(work / block) blocks), which measured faster on gfx950 than
// fewer blocks striding over the array; the kernels keep a grid-stride loop
// only for work beyond max_blocks * block.
inline unsigned grid_for(uint64_t work, int block, uint64_t max_blocks = 1ull << 30)
{
    // a dispatch holds its grid size in work-items as a 32-bit number
    const uint64_t dispatch_cap = 0xFFFFFFFFull / (uint64_t)block;
    if (max_blocks > dispatch_cap) max_blocks = dispatch_cap;
    uint64_t b = (work + block - 1) / block;
    if (b > max_blocks) b = max_blocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Stages `bytes` of host data into the qureg's device matrix ring and returns
// the device address (ordered on the qureg's stream).
int stage_matrix(qs_qureg *q, const void *host, size_t bytes, const void **dev);

// Device reduction helpers, defined in reduce.hip.
int finish_reduction(qs_qureg *q, int blocks, int width, double *out);
// Doubles of q->d_partials that the Pauli-sum expectation value uses at most.
constexpr size_t kExpecPartials = 2 * (size_t)kReduceBlocks;
// The Pauli-sum expectation value of qs_calc_expec_pauli_sum on q, whose
// d_partials / d_result / h_result serve as its scratch.
int expec_pauli_sum(qs_qureg *q, const int *paulis, const double *coeffs, int num_terms, double *out_re,
                    double *out_im);

// ---- dense gates (gates.hip) ---------------------------------------------------

using cd = std::complex<double>;

enum { kDenseVector = 0, kDenseMfma = 1 };

// Reorders a matrix whose index bit q belongs to targs[q] into ascending
// target order; sorted_out receives the sorted targets.
std::vector<cd> permute_to_sorted(const std::vector<cd> &M, const std::vector<int> &targs,
                                  std::vector<int> &sorted_out);
// Device bytes of a dense matrix in a kernel's layout (0: passed by value).
size_t dense_matrix_bytes(int precision, int nt, int kernel);
// Writes Ms (ascending target order, FP64) into out in the kernel's layout.
void pack_dense(int precision, int nt, int kernel, const std::vector<cd> &Ms, void *out);
// Kernel family used for an nt-target dense gate at a precision.
int choose_dense_kernel(int precision, int nt);
// Launches a dense gate whose matrix Ms is in ascending target order; dev is
// its device copy in the kernel's layout, or null to stage it now.
int launch_dense(qs_qureg *q, const std::vector<int> &ctrls, const std::vector<int> &sorted_targs,
                 const std::vector<cd> &Ms, const void *dev, int kernel);
int apply_raw_gate(qs_qureg *q, const std::vector<int> &ctrls, const std::vector<int> &targs,
                   const std::vector<cd> &M);
int apply_raw_gadget(qs_qureg *q, const std::vector<int> &targs, const std::vector<int> &paulis, double theta);
// rho -> G rho G^dagger for the Pauli gadget G on a density matrix, one pass
// (special.hip).
int apply_density_gadget(qs_qureg *q, const int *targs, const int *paulis, int num_targs, double theta);
std::vector<cd> superop_of_kraus(const std::vector<std::vector<cd>> &ks, int n);

// ---- tuning knobs (tune.hip) ---------------------------------------------------

// 1: dense gates of 4-6 targets on complex64 use MFMA, 0: vector FMAs.
int mfma_preference();
// Upper bound on the MFMA kernel's grid for a k-target gate.
uint64_t mfma_block_cap(int k);

// Tile-step grids for tiles of 2^tile_d amplitudes: resident blocks each
// walking a run of consecutive tiles, resident blocks walking tiles
// blockIdx + k gridDim, or one block per tile.
enum { kTileGridChunk = 0, kTileGridStride = 1, kTileGridPerTile = 2 };
int tile_grid_policy(int tile_d);
// Tiles per block under the chunk policy (0: as many blocks as stay resident).
uint64_t tile_chunk();
// Waves per SIMD that specialised tile steps are compiled for (bounds their
// registers).
int step_waves_per_eu(bool f32);

// Number of lowest qubits every tile step holds (a tile is read in runs of
// 2^this amplitudes).
int tile_low_qubits(int precision);

// Key of a recorded circuit's contents (circuit.hip).
uint64_t circuit_fingerprint(const qs_circuit *c);
int circuit_num_qubits(const qs_circuit *c);

}  // namespace qs
