// Recorded circuits shared by the fusion planner (circuit.hip) and the LDS
// tile engine (tiles.hip).
#pragma once

#include "common.hpp"

namespace qs {

struct CircOp {
    bool gadget;
    std::vector<int> ctrls, targs;    // unitary: controls, targets in matrix order
    std::vector<cd> M;                // unitary matrix, row-major 2^nt x 2^nt
    std::vector<int> paulis;          // gadget: codes per target
    double theta;
    std::vector<int> support() const
    {
        std::vector<int> s;
        if (gadget) {
            for (size_t k = 0; k < targs.size(); k++)
                if (paulis[k] != 0) s.push_back(targs[k]);
        } else {
            s = ctrls;
            s.insert(s.end(), targs.begin(), targs.end());
        }
        return s;
    }
};

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

struct Pass {
    bool gadget;
    std::vector<int> ctrls, sorted_targs;
    std::vector<cd> Ms;               // dense matrix in ascending target order
    std::vector<int> gtargs, paulis;  // gadget pass
    double theta;
    int kernel;
    size_t dev_offset;                // into the circuit's device buffer
    bool has_dev;
    int members;
    // LDS tile step
    bool tile = false;
    int tile_d = 0;
    std::vector<uint64_t> basis;      // w_k by coordinate
    std::vector<int> pivots;          // pivot bit of w_k
    std::vector<RPhase> phases;
    std::vector<ROp> rops;
    std::vector<cd> tmats;            // dense matrices of the step, concatenated
};

// LDS tile engine (tiles.hip).
// Largest tile dimension usable for a precision on this device.
int tile_dim_limit(int precision);
// Plans the circuit as LDS tile steps of at most T dimensions (operators
// that do not fit a tile become single passes) into c->passes.
void plan_tiles(qs_circuit *c, int T, int precision);
size_t tile_pass_bytes(const Pass &p, int precision);
void pack_tile_pass(const Pass &p, int precision, void *out);
int launch_tile_pass(qs_qureg *q, const Pass &p, const void *dev);

Pass single_pass(const CircOp &op);

}  // namespace qs

struct qs_circuit {
    int num_qubits;
    int is_density = 0;    // ops act on the Choi vector of an N-qubit density matrix
    int index_bits = 0;    // N, or 2N for a density circuit: the qubits ops address
    std::vector<qs::CircOp> ops;
    std::vector<qs::Pass> passes;
    bool compiled = false;
    int precision = -1;
    int fuse_k = 0;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int device = -1;
};
