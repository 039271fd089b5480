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

constexpr int kTileDimMax = 14;

// One operator of an LDS tile step, in the tile's coordinates.  The tile is
// the coset base ^ span(w_0..w_{d-1}) (reduced echelon basis, coordinate k
// <-> w_k in ascending pivot order); element c sits at base ^ (xor of w_k
// over the set bits k of c), and qubit b of element c equals
// bit b of base ^ parity(c & m_b), m_b = sum_k (bit b of w_k) << k.
struct TOp {
    int kind;            // 0: dense gate on unit-vector coordinates, 1: Pauli gadget
    int nt, nc;          // dense: targets, controls
    int pos[3];          // dense: target coordinates, ascending
    int cq[4];           // dense: control qubits
    uint32_t cm[4];      // dense: control coordinate masks m_c
    uint32_t flip;       // gadget: coordinate flip of its X/Y mask (0: diagonal)
    uint32_t yzm;        // gadget: xor of m_b over its Y/Z qubits
    uint64_t yz;         // gadget: Y/Z qubit mask
    int mat;             // dense: first entry of its matrix in the pass's table
    double cs, cre, cim; // gadget: cos(theta) and i sin(theta) i^{#Y}
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
    std::vector<TOp> tops;
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
    std::vector<qs::CircOp> ops;
    std::vector<qs::Pass> passes;
    bool compiled = false;
    int precision = -1;
    int fuse_k = 0;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int device = -1;
};
