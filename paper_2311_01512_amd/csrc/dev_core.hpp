// Definitions shared by the device code of the library and by the tile-step
// kernels compiled at run time: amplitude types, bit insertion, the
// register-phase and operator records of tile steps.  The library embeds this
// header and tile_dev.hpp as text for the run-time compilation.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qs {

template <typename A, typename B> struct same_type { static constexpr bool value = false; };
template <typename A> struct same_type<A, A> { static constexpr bool value = true; };

// ---- amplitudes --------------------------------------------------------------

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using C2 = typename cplx_t<R>::type;

template <typename R> __device__ __forceinline__ C2<R> mk(R x, R y) { C2<R> c; c.x = x; c.y = y; return c; }

// acc += m * v (complex)
template <typename R>
__device__ __forceinline__ void cmac(C2<R> &acc, const C2<R> m, const C2<R> v)
{
    acc.x = fma(m.x, v.x, acc.x);
    acc.x = fma(-m.y, v.y, acc.x);
    acc.y = fma(m.x, v.y, acc.y);
    acc.y = fma(m.y, v.x, acc.y);
}

template <typename R>
__device__ __forceinline__ C2<R> cmul(const C2<R> a, const C2<R> b)
{
    return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- bit-index algebra (Alg. "bit_twiddles") ------------------------------------

constexpr int kMaxInsert = 24;   // qubits spliced into a loop index by one launch

// Splices zero bits into an index at ascending positions q_0 < q_1 < ...
// (insertBits of the paper with b = 0), stored as the masks (1 << q_k) - 1.
struct InsertPlan {
    int n;
    uint64_t low[kMaxInsert];
};

__device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const InsertPlan &p)
{
#pragma unroll 4
    for (int k = 0; k < p.n; k++) {
        const uint64_t lo = p.low[k];
        g = (g & lo) | ((g & ~lo) << 1);
    }
    return g;
}

// Tile steps.  A tile is the coset base ^ span(w_0..w_{d-1}) (reduced
// echelon basis, coordinate k <-> w_k in ascending pivot order); element c
// sits at base ^ (xor of w_k over the set bits k of c), and qubit b of
// element c equals bit b of base ^ parity(c & m_b), m_b = sum_k (bit b of
// w_k) << k.  Each thread of the block holds kRegs elements of the tile in
// registers; which elements is the layout of a phase (RPhase), and every
// operator of a phase only mixes elements held by one thread.
constexpr int kRegBits = 3;
constexpr int kRegs = 1 << kRegBits;
constexpr int kTileDimMax = kRegBits + 10;   // 1024 threads per block

// Thread t holds coordinates tau(t) ^ rho[u], u < kRegs: rho spans the
// phase's register subspace (basis r_j, each with its own pivot bit), and
// tau deposits the bits of t, in order, at the coordinates that are not
// pivots.  In a phase with matrix-core operators (c4 >= 0) bits 4 and 5 of t
// go to the lane coordinates c4 and c5 instead, and the other bits skip them.
struct RPhase {
    uint32_t rho[kRegs];
    uint32_t lo[kRegBits + 2];      // (1 << q) - 1 for the pivots and lane coordinates, ascending
    int nlo;                        // kRegBits, or kRegBits + 2 with lane coordinates
    int c4, c5;
    uint32_t pad_;
    uint64_t yaddr[kRegs];          // index offset of rho[u] (xor of w_k)
    uint64_t taddr[kTileDimMax];    // index offset of thread bit k
    int first_op, num_ops;
};

// One operator of a phase, on register indices.
//   code 1..7: dense gate whose targets are the register bits set in code
//              (matrix bit i <-> i-th lowest of them); 17..23: the same with
//              nc controls, control i set where bit cq[i] of base ^
//              parity(tau & cm[i]) ^ bit i of qtab's nibble u is 1
//   code 8:    diagonal Pauli gadget; code 9..15: gadget pairing register u
//              with u ^ (code - 8).  Sign parity of element (t, u) is
//              parity(base & yz) ^ parity(tau & yzm) ^ parity(u & gy); the
//              partner's sign is folded into (pre, pim).
//   code 32..38: dense gate on the matrix cores (complex64): targets on the
//              lane coordinates c4, c5 and the register bits set in code - 32;
//              mat indexes its per-lane MFMA coefficients; controls as above.
//   code 16:   multiplies every amplitude by cs (the step's gadget factors
//              when no matrix of the step took them).
//   code 24..31 / 40..47: gadget with cos(theta) factored out, pairing
//              register u with u ^ (code - 24) / u ^ (code - 40) (24: the
//              diagonal Z-only case); the partner term is cre u (resp. pre u)
//              times the sign, u = i for codes 24..31 and 1 for 40..47.
//   code 64 + 4 UM + s: uncontrolled gate on register bits UM (1 or 2 of
//              them) whose matrix couples member j only with j ^ s (s = 0:
//              diagonal).
struct ROp {
    int code;
    int nc;
    int cq[4];
    uint32_t cm[4];
    uint64_t qtab;
    uint64_t yz;
    uint32_t yzm, gy;
    int mat;                        // first entry of its matrix in the table
    uint32_t hsel;                  // matrix-core gate: 2 bits per register, rho[u] at (c4, c5)
    double cs, cre, cim;            // gadget: cos(theta), i sin(theta) i^{#Y}
    double pre, pim;                // (cre, cim) times (-1)^parity(x & yz)
    float fcs, fcre, fcim, fpre, fpim;   // the same in FP32 for complex64 tiles
};

}  // namespace qs
