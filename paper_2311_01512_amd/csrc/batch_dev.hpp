// Device code of the batch's register-phase path (batch.hip), shared with
// the step kernels that qs_batch_specialize compiles at run time: the
// device tables, the per-operator register arithmetic and the LDS exchange
// between phases.  A specialised kernel hands compile-time operator records
// to the same functions as the generic kernels, so both compute the same
// values.  The library embeds this header as text for the run-time
// compilation.
#pragma once

#include "dev_core.hpp"

namespace qs {

constexpr int kTileMax = 12;

enum { BOP_ROT = 0, BOP_GATE = 1, BOP_CZ = 2 };

// Device descriptors.
struct DOp {
    int kind;
    int pos0, pos1;   // positions of q0 / q1 inside the step's qubit set, -1 if outside
    int q0, q1;
    int pauli;
    int param;        // global parameter index (rotations)
    int grad;         // rotation slot, -1 for other operators
    uint64_t gpart;   // first gradient partial of this rotation (one per tile)
    int rbit;         // register bit of a 1-qubit operator in its phase (register path); for
                      // a CZ, of q0, or -1 where q0 is not a register coordinate
    int rbit1;        // a CZ's register bit of q1, or -1
    int czrun;        // register path, CZ: bit 0 first, bit 1 last of a run of CZs in its phase
    int slot;         // gradient slot of a rotation within its phase (register path)
    double scale;
    double m[8];      // fixed gate, row-major (re, im)
};

struct DStep {
    uint64_t amp_off;
    InsertPlan plan;  // zeros at the step's qubits: spreads the tile number
    int qn;
    int qpos[kTileMax];
    int op_begin, op_end;
    int ph_begin, ph_end;   // register phases (steps of >= kRegMinQubits qubits)
    int prog;               // specialised step program of a register-path step (-1: none)
    int first;              // step 0 of its circuit: reads |0..0> instead of the state
};

// Amplitude o of a circuit's state at the start of a step: for a circuit's
// first step the initial state |0..0> (every run starts from it), so that no
// launch has to write it first.
template <typename R>
__device__ __forceinline__ C2<R> load_amp(const C2<R> *__restrict__ a, uint64_t o, bool zero_state)
{
    if (zero_state) return mk<R>(o == 0 ? R(1) : R(0), R(0));
    return a[o];
}

// Register phases of a step (tiles of at least 2^kRegMinQubits amplitudes):
// thread t of the block holds the 8 tile coordinates tau(t) | rho(u), where
// rho puts the bits of u on the coordinates rc[0..2] and tau deposits the
// bits of t, in order, on the others (zeros inserted at lo).  Every 1-qubit
// operator of the phase acts on one of the rc coordinates, so it only mixes
// registers of one thread; CZ is diagonal and needs none.  The tile moves
// through LDS once per phase change.
constexpr int kRegMinQubits = 9;     // 64 threads: whole wavefronts
constexpr int kPhaseRotMax = 32;     // gradient slots per phase
struct BPhase {
    uint32_t lo[3];                  // (1 << rc) - 1, ascending
    int rc[3];                       // coordinate of register bit j
    int op_begin, op_end;
};

// v moved across lanes by a DPP control (both 32-bit halves); lanes of rows
// outside row_mask receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v)
{
    int lo, hi;
    __builtin_memcpy(&lo, &v, 4);
    __builtin_memcpy(&hi, reinterpret_cast<const char *>(&v) + 4, 4);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
    double r;
    __builtin_memcpy(&r, &lo, 4);
    __builtin_memcpy(reinterpret_cast<char *>(&r) + 4, &hi, 4);
    return r;
}

// Sum over the active lanes of the wavefront, returned to every lane, with
// data-parallel primitive moves instead of LDS permutes: within each row of
// 16 lanes by quad permutes and mirrors (every lane ends with its row's
// sum), then across rows by the row broadcasts of lanes 15 and 31 (the last
// lane ends with the total).  Moves from inactive lanes bring 0, so for the
// active sets used here, a prefix of 2^k lanes, the last active lane holds
// the total and is read back.
__device__ __forceinline__ double bwave_sum(double v)
{
    v += dpp_move<0xB1>(v);        // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);        // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);       // row_half_mirror
    v += dpp_move<0x140>(v);       // row_mirror
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    int lo, hi;
    __builtin_memcpy(&lo, &v, 4);
    __builtin_memcpy(&hi, reinterpret_cast<const char *>(&v) + 4, 4);
    const int last = 63 - __builtin_clzll(__builtin_amdgcn_read_exec());
    lo = __builtin_amdgcn_readlane(lo, last);
    hi = __builtin_amdgcn_readlane(hi, last);
    double r;
    __builtin_memcpy(&r, &lo, 4);
    __builtin_memcpy(reinterpret_cast<char *>(&r) + 4, &hi, 4);
    return r;
}

// v moved within rows of 16 lanes by a DPP control whose every lane has a
// source lane in its row (quad permutes, mirrors): no old value is kept.
template <int CTRL>
__device__ __forceinline__ double dpp_row_move(double v)
{
    int lo, hi;
    __builtin_memcpy(&lo, &v, 4);
    __builtin_memcpy(&hi, reinterpret_cast<const char *>(&v) + 4, 4);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    double r;
    __builtin_memcpy(&r, &lo, 4);
    __builtin_memcpy(reinterpret_cast<char *>(&r) + 4, &hi, 4);
    return r;
}

// Sum over each row of 16 lanes (every lane of the row receives it), all
// lanes active: quad permutes and mirrors as in bwave_sum.
__device__ __forceinline__ double brow_sum(double v)
{
    v += dpp_row_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_row_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_row_move<0x141>(v);   // row_half_mirror
    v += dpp_row_move<0x140>(v);   // row_mirror
    return v;
}

// Partial sums of a phase's rotations: one per row of 16 lanes (4 per
// wavefront, 8 wavefronts at most) and gradient slot.
constexpr int kRedRows = 32;

// 2 x 2 matrix of an operator; dir = -1 gives its adjoint.  A rotation's
// cos and sin come from the per-operator table trig (filled by k_batch_trig
// for the current parameters), not from a per-lane sincos.
template <typename R>
__device__ __forceinline__ void op_matrix(const DOp &op, const double *trig, int dir, C2<R> (&u)[4])
{
    if (op.kind == BOP_ROT) {
        const double c = trig[0], s = dir * trig[1];
        if (op.pauli == 1) {          // c 1 + i s X
            u[0] = mk<R>(c, 0); u[1] = mk<R>(0, s); u[2] = mk<R>(0, s); u[3] = mk<R>(c, 0);
        } else if (op.pauli == 2) {   // c 1 + i s Y
            u[0] = mk<R>(c, 0); u[1] = mk<R>(s, 0); u[2] = mk<R>(-s, 0); u[3] = mk<R>(c, 0);
        } else {                      // c 1 + i s Z
            u[0] = mk<R>(c, s); u[1] = mk<R>(0, 0); u[2] = mk<R>(0, 0); u[3] = mk<R>(c, -s);
        }
    } else if (dir > 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) u[k] = mk<R>((R)op.m[2 * k], (R)op.m[2 * k + 1]);
    } else {                          // conjugate transpose
        u[0] = mk<R>((R)op.m[0], (R)-op.m[1]);
        u[1] = mk<R>((R)op.m[4], (R)-op.m[5]);
        u[2] = mk<R>((R)op.m[2], (R)-op.m[3]);
        u[3] = mk<R>((R)op.m[6], (R)-op.m[7]);
    }
}

// ---- register-phase path (tiles of >= 2^kRegMinQubits amplitudes) ----------------------

__device__ __forceinline__ uint32_t bphase_tau(uint32_t t, const BPhase &ph)
{
#pragma unroll
    for (int b = 0; b < 3; b++) {
        const uint32_t lo = ph.lo[b];
        t = (t & lo) | ((t & ~lo) << 1);
    }
    return t;
}

__device__ __forceinline__ uint32_t bphase_rho(int u, const BPhase &ph)
{
    return ((uint32_t)(u & 1) << ph.rc[0]) | ((uint32_t)((u >> 1) & 1) << ph.rc[1]) |
           ((uint32_t)((u >> 2) & 1) << ph.rc[2]);
}

// 2 x 2 matrix (m0 m1; m2 m3) on the register pairs (u0, u0 | 1 << J).
template <typename R, int J>
__device__ __forceinline__ void reg_pairs(C2<R> (&x)[8], C2<R> m0, C2<R> m1, C2<R> m2, C2<R> m3)
{
#pragma unroll
    for (int u0 = 0; u0 < 8; u0++) {
        if ((u0 >> J) & 1) continue;
        const C2<R> a = x[u0], b = x[u0 | (1 << J)];
        C2<R> p = mk<R>(0, 0), q = mk<R>(0, 0);
        cmac<R>(p, m0, a);
        cmac<R>(p, m1, b);
        cmac<R>(q, m2, a);
        cmac<R>(q, m3, b);
        x[u0] = p;
        x[u0 | (1 << J)] = q;
    }
    // a distinct empty statement per J: keeps the compiler from sinking the
    // three dispatch arms of reg_gate into one, which would address the
    // registers through pointers (private memory)
    if constexpr (J == 0) asm volatile("; reg pairs 0");
    else if constexpr (J == 1) asm volatile("; reg pairs 1");
    else asm volatile("; reg pairs 2");
}

// Partial of Im <lambda|P|phi> over the register pairs (u0, u0 | 1 << J) of a
// rotation exp(i theta P) on register bit J.
template <typename R, int J>
__device__ __forceinline__ double reg_grad_pairs(const C2<R> (&x)[8], const C2<R> (&y)[8], int pauli)
{
#pragma clang fp contract(off)
    double im = 0.0;
#pragma unroll
    for (int u0 = 0; u0 < 8; u0++) {
        if ((u0 >> J) & 1) continue;
        const int u1 = u0 | (1 << J);
        const C2<R> f0 = x[u0], f1 = x[u1], l0 = y[u0], l1 = y[u1];
        C2<R> p0, p1;   // (P phi) at the two members
        if (pauli == 1) {
            p0 = f1;
            p1 = f0;
        } else if (pauli == 2) {   // Y: -i phi_1 at member 0, +i phi_0 at member 1
            p0 = mk<R>(f1.y, -f1.x);
            p1 = mk<R>(-f0.y, f0.x);
        } else {
            p0 = f0;
            p1 = mk<R>(-f1.x, -f1.y);
        }
        // complex64 states: the pair's products in FP32 (relative error about
        // 1e-7, below the states' own), the sums over lanes, waves and tiles
        // in FP64.  Explicit FMAs, so that every build rounds alike.
        R v = -(l1.y * p1.x);
        v = fma(l1.x, p1.y, v);
        v = fma(-l0.y, p0.x, v);
        v = fma(l0.x, p0.y, v);
        if (u0 == 0) im = (double)v;   // the first pair (u0 = 0 never has bit J)
        else im += (double)v;
    }
    if constexpr (J == 0) asm volatile("; grad pairs 0");
    else if constexpr (J == 1) asm volatile("; grad pairs 1");
    else asm volatile("; grad pairs 2");
    return im;
}

// Rotation c 1 + i s P (P = X, Y, Z by PA = 1, 2, 3) on the register pairs
// (u0, u0 | 1 << J): the matrix's zeros and its real or imaginary entries
// spelled out, 8 FP operations per pair instead of a general 2 x 2
// complex product's 16.  Explicit FMAs (no implicit contraction), so that
// the generic kernels and the specialised ones round alike.
template <typename R, int J, int PA>
__device__ __forceinline__ void reg_rot_pairs(C2<R> (&x)[8], R c, R s)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int u0 = 0; u0 < 8; u0++) {
        if ((u0 >> J) & 1) continue;
        const C2<R> a = x[u0], b = x[u0 | (1 << J)];
        if constexpr (PA == 1) {          // (c a + i s b, i s a + c b)
            x[u0] = mk<R>(fma(c, a.x, -(s * b.y)), fma(c, a.y, s * b.x));
            x[u0 | (1 << J)] = mk<R>(fma(c, b.x, -(s * a.y)), fma(c, b.y, s * a.x));
        } else if constexpr (PA == 2) {   // (c a + s b, c b - s a)
            x[u0] = mk<R>(fma(c, a.x, s * b.x), fma(c, a.y, s * b.y));
            x[u0 | (1 << J)] = mk<R>(fma(c, b.x, -(s * a.x)), fma(c, b.y, -(s * a.y)));
        } else {                          // ((c + i s) a, (c - i s) b)
            x[u0] = mk<R>(fma(c, a.x, -(s * a.y)), fma(c, a.y, s * a.x));
            x[u0 | (1 << J)] = mk<R>(fma(c, b.x, s * b.y), fma(c, b.y, -(s * b.x)));
        }
    }
    // distinct empty statements, as in reg_pairs
    if constexpr (J == 0) asm volatile("; rot pairs 0");
    else if constexpr (J == 1) asm volatile("; rot pairs 1");
    else asm volatile("; rot pairs 2");
}

template <typename R, int PA>
__device__ __forceinline__ void reg_rot_p(C2<R> (&x)[8], int rbit, R c, R s)
{
    switch (rbit) {
    case 0: reg_rot_pairs<R, 0, PA>(x, c, s); break;
    case 1: reg_rot_pairs<R, 1, PA>(x, c, s); break;
    default: reg_rot_pairs<R, 2, PA>(x, c, s); break;
    }
}

// A rotation exp(i theta P) (s = dir sin(theta)) on register bit rbit.
template <typename R>
__device__ __forceinline__ void reg_rot(C2<R> (&x)[8], int rbit, int pauli, R c, R s)
{
    if (pauli == 1) reg_rot_p<R, 1>(x, rbit, c, s);
    else if (pauli == 2) reg_rot_p<R, 2>(x, rbit, c, s);
    else reg_rot_p<R, 3>(x, rbit, c, s);
}

template <typename R>
__device__ __forceinline__ void reg_gate(C2<R> (&x)[8], int rbit, const C2<R> (&u)[4])
{
    switch (rbit) {
    case 0: reg_pairs<R, 0>(x, u[0], u[1], u[2], u[3]); break;
    case 1: reg_pairs<R, 1>(x, u[0], u[1], u[2], u[3]); break;
    default: reg_pairs<R, 2>(x, u[0], u[1], u[2], u[3]); break;
    }
}

// CZ on the register path.  Which of a thread's 8 registers a CZ negates is
// an 8-bit mask over u: a qubit held in register bit j selects the registers
// with bit j of u set (0xAA, 0xCC, 0xF0), a qubit on a thread coordinate is 1
// for all 8 registers or none, a qubit outside the tile reads the tile's base
// bit; the CZ negates where both are 1.  CZs are diagonal and commute with
// each other, so a run of them is one mask (the xor of theirs) and one pass
// of sign flips.
__device__ __forceinline__ uint32_t cz_side(int pos, int rb, int q, uint32_t tau, uint64_t base)
{
    if (rb >= 0) return rb == 0 ? 0xAAu : (rb == 1 ? 0xCCu : 0xF0u);
    if (pos >= 0) return 0u - ((tau >> pos) & 1u);
    return ((base >> q) & 1ULL) ? 0xFFu : 0u;
}

__device__ __forceinline__ uint32_t cz_mask(const DOp &op, uint32_t tau, uint64_t base)
{
    return cz_side(op.pos0, op.rbit, op.q0, tau, base) & cz_side(op.pos1, op.rbit1, op.q1, tau, base);
}

__device__ __forceinline__ float flip_sign(float v, uint32_t s) { return __uint_as_float(__float_as_uint(v) ^ s); }

__device__ __forceinline__ double flip_sign(double v, uint32_t s)
{
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)((uint64_t)s << 32));
}

// Negates register u where bit u of mask is set (the sign bit flipped).
template <typename R>
__device__ __forceinline__ void reg_sign(C2<R> (&x)[8], uint32_t mask)
{
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t s = (mask << (31 - u)) & 0x80000000u;
        x[u] = mk<R>(flip_sign(x[u].x, s), flip_sign(x[u].y, s));
    }
}

// Global offset of tile coordinates c (deposited at the step's qubits).
__device__ __forceinline__ uint64_t tile_offset_bits(uint32_t c, const DStep &st)
{
    uint64_t o = 0;
    for (int b = 0; b < st.qn; b++) o |= (uint64_t)((c >> b) & 1u) << st.qpos[b];
    return o;
}

// Global offsets of the 8 registers of a phase: the qubits of rc[j] for the
// bits j of u (no loops, so register indices stay compile-time).
struct RegOffsets {
    uint64_t q[3];
    __device__ __forceinline__ RegOffsets(const BPhase &ph, const DStep &st)
    {
#pragma unroll
        for (int j = 0; j < 3; j++) q[j] = 1ULL << st.qpos[ph.rc[j]];
    }
    __device__ __forceinline__ uint64_t operator()(int u) const
    {
        return ((u & 1) ? q[0] : 0ULL) | ((u & 2) ? q[1] : 0ULL) | ((u & 4) ? q[2] : 0ULL);
    }
};

// LDS exchange between the register layouts of phases Q and P: every thread
// of the block takes part in the barriers; active threads write their
// registers in Q's layout and read them back in P's.  Returns P's tau.
template <typename R>
__device__ __forceinline__ uint32_t bphase_exchange(C2<R> (&x)[8], C2<R> *v, uint32_t tau, const BPhase &Q,
                                                    const BPhase &P, bool active)
{
    const uint32_t tn = bphase_tau(threadIdx.x, P);
    __syncthreads();   // earlier reads of the LDS tile are done
    if (active) {
#pragma unroll
        for (int u = 0; u < 8; u++) v[tau | bphase_rho(u, Q)] = x[u];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int u = 0; u < 8; u++) x[u] = v[tn | bphase_rho(u, P)];
    }
    return tn;
}

// The same for the two tiles (phi, lambda) of the adjoint sweep.
template <typename R>
__device__ __forceinline__ uint32_t bphase_exchange2(C2<R> (&x)[8], C2<R> (&y)[8], C2<R> *vphi, C2<R> *vlam,
                                                     uint32_t tau, const BPhase &Q, const BPhase &P, bool active)
{
    const uint32_t tn = bphase_tau(threadIdx.x, P);
    if (active) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint32_t c = tau | bphase_rho(u, Q);
            vphi[c] = x[u];
            vlam[c] = y[u];
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint32_t c = tn | bphase_rho(u, P);
            x[u] = vphi[c];
            y[u] = vlam[c];
        }
    }
    return tn;
}

// Operator k (global index; trig holds its cos and sin) of a forward phase.
// czm carries the sign mask of a run of CZs until the run's last one.
template <typename R>
__device__ __forceinline__ void fwd_op(C2<R> (&x)[8], const DOp &op, int k, const double *__restrict__ trig,
                                       uint32_t tau, uint64_t base, uint32_t &czm)
{
    if (op.kind == BOP_CZ) {
        czm ^= cz_mask(op, tau, base);
        if (op.czrun & 2) {   // the run's last CZ
            reg_sign<R>(x, czm);
            czm = 0;
        }
    } else if (op.kind == BOP_ROT) {
        reg_rot<R>(x, op.rbit, op.pauli, (R)trig[2 * k], (R)trig[2 * k + 1]);
    } else {
        C2<R> u[4];
        op_matrix<R>(op, trig + 2 * k, +1, u);
        reg_gate<R>(x, op.rbit, u);
    }
}

// Operator k of the adjoint sweep (operators last first): a rotation's
// partial Im <lambda|P|phi> over the thread's register pairs, summed over
// each row of 16 lanes into red[slot][4 wave + row], then U^dagger on both
// tiles.  czm as
// in fwd_op, applied at the run's first CZ (reached last).
template <typename R>
__device__ __forceinline__ void bwd_op(C2<R> (&x)[8], C2<R> (&y)[8], const DOp &op, int k,
                                       const double *__restrict__ trig, uint32_t tau, uint64_t base, uint32_t &czm,
                                       double (*red)[kRedRows], int lane, int wave)
{
    if (op.kind == BOP_CZ) {
        czm ^= cz_mask(op, tau, base);
        if (op.czrun & 1) {   // the run's first CZ, reached last
            reg_sign<R>(x, czm);
            reg_sign<R>(y, czm);
            czm = 0;
        }
        return;
    }
    if (op.grad >= 0) {
        double im;
        switch (op.rbit) {
        case 0: im = reg_grad_pairs<R, 0>(x, y, op.pauli); break;
        case 1: im = reg_grad_pairs<R, 1>(x, y, op.pauli); break;
        default: im = reg_grad_pairs<R, 2>(x, y, op.pauli); break;
        }
        im = brow_sum(im);
        if ((lane & 15) == 15) red[op.slot][4 * wave + (lane >> 4)] = im;
    }
    if (op.kind == BOP_ROT) {
        const R c = (R)trig[2 * k], sn = -(R)trig[2 * k + 1];   // the adjoint
        reg_rot<R>(x, op.rbit, op.pauli, c, sn);
        reg_rot<R>(y, op.rbit, op.pauli, c, sn);
    } else {
        C2<R> u[4];
        op_matrix<R>(op, trig + 2 * k, -1, u);
        reg_gate<R>(x, op.rbit, u);
        reg_gate<R>(y, op.rbit, u);
    }
}

// Thread 0.. of the block: the rotation partials of the finished phase
// [op_begin, op_end) summed over the rows of the wavefronts (fixed order)
// into gpart, one thread per operator.
__device__ __forceinline__ void flush_phase(const DOp *__restrict__ ops, int op_begin, int op_end,
                                            const double (*red)[kRedRows], int nwaves, uint32_t tile,
                                            double *__restrict__ gpart)
{
    for (int i = (int)threadIdx.x; i < op_end - op_begin; i += (int)blockDim.x) {
        const DOp &op = ops[op_begin + i];
        if (op.grad < 0) continue;
        double v = 0.0;
        for (int w = 0; w < 4 * nwaves; w++) v += red[op.slot][w];
        gpart[op.gpart + tile] = v;
    }
}

}  // namespace qs
