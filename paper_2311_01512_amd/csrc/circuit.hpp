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
    int param = -1;                   // parametrised gadget: theta = scale * params[param]
    double scale = 1.0;
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

// Qubit masks of a recorded operator for commutation tests: a gadget as its
// Pauli string X^x Z^z (Y sets both), a unitary as its targets and controls.
struct OpMasks {
    bool gadget = false;
    uint64_t x = 0, z = 0, t = 0, c = 0;
};

inline OpMasks op_masks(const CircOp &op)
{
    OpMasks m;
    m.gadget = op.gadget;
    if (op.gadget) {
        for (size_t k = 0; k < op.targs.size(); k++) {
            const uint64_t b = 1ULL << op.targs[k];
            if (op.paulis[k] == 1 || op.paulis[k] == 2) m.x |= b;
            if (op.paulis[k] == 2 || op.paulis[k] == 3) m.z |= b;
        }
    } else {
        for (int q : op.targs) m.t |= 1ULL << q;
        for (int q : op.ctrls) m.c |= 1ULL << q;
    }
    return m;
}

// Whether the two operators commute (a sufficient test): Pauli gadgets when
// their strings commute (an even number of qubits where they anticommute);
// a gadget and a gate when the gadget is the identity on the gate's targets
// and the identity or Z on its controls; two gates when no target of either
// is a qubit of the other (shared controls commute).
inline bool ops_commute(const OpMasks &a, const OpMasks &b)
{
    if (a.gadget && b.gadget) return (__builtin_popcountll((a.x & b.z) ^ (a.z & b.x)) & 1) == 0;
    if (a.gadget || b.gadget) {
        const OpMasks &g = a.gadget ? a : b, &u = a.gadget ? b : a;
        return ((g.x | g.z) & u.t) == 0 && (g.x & u.c) == 0;
    }
    return (a.t & (b.t | b.c)) == 0 && (b.t & a.c) == 0;
}

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
    // kernel specialised for this step at run time (jit.hip), or null
    void *jit_fn = nullptr;
    unsigned jit_grid = 0;            // its resident-block grid
    unsigned jit_lds = 0;             // its dynamic LDS bytes (tile, then staged tables)
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
// Offset of a tile pass's matrix table within its device tables.
size_t tile_mats_offset(const Pass &p);
// Run-time specialisation of a compiled circuit's tile steps (jit.hip).
int specialize_tiles(qs_circuit *c, int *num_kernels);
// HIP sources -> code objects for `arch` (rtc.hip): from the process cache,
// the disk cache, or the ROCm clang in parallel child processes.
int compile_device_sources(const std::vector<std::string> &srcs, const std::string &arch,
                           std::vector<std::vector<char>> &codes);
void release_specialized(qs_circuit *c);
// Records that passes of c were queued on stream s (after them), and waits
// for every such use to finish (before tables or kernels are released).
int note_circuit_use(qs_circuit *c, hipStream_t s);
void wait_circuit_uses(qs_circuit *c);

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
    std::vector<void *> jit_modules;   // modules of the specialised tile-step kernels
    // one event per stream the circuit's passes were queued on, recorded after
    // the last of them: tables and kernels are released only once they passed
    std::vector<std::pair<void *, void *>> uses;   // (hipStream_t, hipEvent_t)
};
