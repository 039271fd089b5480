// Device code of tile steps: the register operators and the phase
// bookkeeping, used by the generic tile-step kernel (tiles.hip) and by the
// per-step kernels compiled at run time from generated source (jit.hip).
#pragma once

#include "dev_core.hpp"

// No implicit fusion of a multiply into an add for the rest of the
// translation unit: the fused operations are the explicit fma calls, so the
// generic kernel and a step compiled with its operators as constants round
// alike (with contraction on, constants let the compiler fuse a different
// product of the same expression).
#pragma clang fp contract(off)

namespace qs {

// i-th lowest set bit of mask receives bit i of l
__host__ __device__ constexpr int deposit_bits(int l, int mask)
{
    int r = 0, k = 0;
    for (int b = 0; b < kRegBits; b++)
        if ((mask >> b) & 1) {
            if ((l >> k) & 1) r |= 1 << b;
            k++;
        }
    return r;
}

__host__ __device__ constexpr int popcount_c(int m) { return m ? (m & 1) + popcount_c(m >> 1) : 0; }

__device__ __forceinline__ uint32_t tau_of(uint32_t t, const RPhase &ph)
{
    if (ph.nlo == kRegBits) {
#pragma unroll
        for (int b = 0; b < kRegBits; b++) {
            const uint32_t lo = ph.lo[b];
            t = (t & lo) | ((t & ~lo) << 1);
        }
        return t;
    }
    uint32_t c = (t & 15u) | ((t >> 6) << 4);
#pragma unroll
    for (int b = 0; b < kRegBits + 2; b++) {
        const uint32_t lo = ph.lo[b];
        c = (c & lo) | ((c & ~lo) << 1);
    }
    return c | (((t >> 4) & 1u) << ph.c4) | (((t >> 5) & 1u) << ph.c5);
}

__device__ __forceinline__ uint64_t thread_offset(uint32_t t, int lb, const RPhase &ph)
{
    uint64_t x = 0;
    for (int k = 0; k < lb; k++)
        if ((t >> k) & 1u) x ^= ph.taddr[k];
    return x;
}

template <typename R, int UM, bool CTRL>
__device__ __forceinline__ void reg_dense(C2<R> (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base,
                                          const C2<R> *__restrict__ m)
{
    constexpr int D = 1 << popcount_c(UM);
    uint32_t tp = 0, full = 0;
    if constexpr (CTRL) {
        for (int i = 0; i < op.nc; i++)
            tp |= (uint32_t)(((base >> op.cq[i]) ^ (uint64_t)__popc(tau & op.cm[i])) & 1ULL) << i;
        full = (1u << op.nc) - 1u;
    }
#pragma unroll
    for (int u0 = 0; u0 < kRegs; u0++) {
        if (u0 & UM) continue;
        // groups whose controls are not all set are left alone; where that
        // holds for a whole wave (controls outside the lane coordinates, the
        // common case) the arithmetic is skipped
        if constexpr (CTRL)
            if ((tp ^ ((uint32_t)(op.qtab >> (4 * u0)) & 15u)) != full) continue;
        C2<R> in[D];
#pragma unroll
        for (int l = 0; l < D; l++) in[l] = x[u0 | deposit_bits(l, UM)];
#pragma unroll
        for (int j = 0; j < D; j++) {
            C2<R> acc = mk<R>(R(0), R(0));
#pragma unroll
            for (int l = 0; l < D; l++) cmac<R>(acc, m[j * D + l], in[l]);
            x[u0 | deposit_bits(j, UM)] = acc;
            // an 8x8 matrix row by row, not all 64 entries in scalar registers
            if constexpr (D == 8) asm volatile("" ::: "memory");
        }
    }
}

// Uncontrolled gate on the register bits UM whose matrix only couples
// member j with j ^ SM (SM = 0: diagonal): one or two complex products per
// amplitude instead of 2^k.
template <typename R, int UM, int SM>
__device__ __forceinline__ void reg_sparse(C2<R> (&x)[kRegs], const C2<R> *__restrict__ m)
{
    constexpr int D = 1 << popcount_c(UM);
#pragma unroll
    for (int u0 = 0; u0 < kRegs; u0++) {
        if (u0 & UM) continue;
        C2<R> in[D];
#pragma unroll
        for (int l = 0; l < D; l++) in[l] = x[u0 | deposit_bits(l, UM)];
#pragma unroll
        for (int j = 0; j < D; j++) {
            C2<R> acc = mk<R>(R(0), R(0));
            cmac<R>(acc, m[j * D + j], in[j]);
            if constexpr (SM != 0) cmac<R>(acc, m[j * D + (j ^ SM)], in[j ^ SM]);
            x[u0 | deposit_bits(j, UM)] = acc;
        }
    }
}

// Element (t, u) has sign parity st ^ parity(u & gy); the pair partner's
// parity differs by parity(x & yz), folded into cre/cim on the host as a
// second constant (ROp::pre/pim) so both outputs use the parity of u0.
template <typename R, int FU>
__device__ __forceinline__ void reg_gadget(C2<R> (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base)
{
    const uint32_t st = (uint32_t)(__popcll(base & op.yz) + __popc(tau & op.yzm)) & 1u;
    const R sg = st ? R(-1) : R(1);
    // uniform constants (scalar registers), in the kernel's precision
    R cs, cr, ci, pr, pi;
    if constexpr (same_type<R, float>::value) {
        cs = op.fcs; cr = op.fcre; ci = op.fcim; pr = op.fpre; pi = op.fpim;
    } else {
        cs = op.cs; cr = op.cre; ci = op.cim; pr = op.pre; pi = op.pim;
    }
    if constexpr (FU == 0) {
        const R kr = sg * cr, ki = sg * ci;   // this thread's sign times i sin(theta) i^{#Y}
        const R ar0 = cs + kr, ar1 = cs - kr, ai1 = -ki;
#pragma unroll
        for (int u = 0; u < kRegs; u++) {
            const bool neg = __popc((uint32_t)u & op.gy) & 1;
            const R ar = neg ? ar1 : ar0, ai = neg ? ai1 : ki;
            const C2<R> a = x[u];
            x[u] = mk<R>(ar * a.x - ai * a.y, ar * a.y + ai * a.x);
        }
    } else {
        constexpr int HB = 31 - __builtin_clz((unsigned)FU);
#pragma unroll
        for (int u0 = 0; u0 < kRegs; u0++) {
            if ((u0 >> HB) & 1) continue;
            const int u1 = u0 ^ FU;
            // sign of (t, u0): this thread's sign times the register parity
            const R s = (__popc((uint32_t)u0 & op.gy) & 1) ? -sg : sg;
            const C2<R> x0 = x[u0], x1 = x[u1];
            // x0' = cs x0 + s(u1) c x1 = cs x0 + s (c (-1)^par(x & yz)) x1,  x1' = cs x1 + s c x0
            const C2<R> t1 = mk<R>(pr * x1.x - pi * x1.y, pr * x1.y + pi * x1.x);
            const C2<R> t0 = mk<R>(cr * x0.x - ci * x0.y, cr * x0.y + ci * x0.x);
            x[u0] = mk<R>(fma(s, t1.x, cs * x0.x), fma(s, t1.y, cs * x0.y));
            x[u1] = mk<R>(fma(s, t0.x, cs * x1.x), fma(s, t0.y, cs * x1.y));
        }
    }
}

// Gadget with cos(theta) factored out into the step's scale: with
// s = this thread's sign times the register parity, k the ratio
// c / cos(theta) as a real number (the imaginary part when IM), u = i (IM)
// or 1:
//   pair:      x0 <- x0 + s kp u x1,  x1 <- x1 + s kc u x0
//   diagonal:  x <- x + s kc i x      (FU = 0, Z only: IM)
// one FMA per real component instead of a complex product.
template <typename R, int FU, bool IM>
__device__ __forceinline__ void reg_gadget_f(C2<R> (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base)
{
    const uint32_t st = (uint32_t)(__popcll(base & op.yz) + __popc(tau & op.yzm)) & 1u;
    R kc, kp;
    if constexpr (same_type<R, float>::value) {
        kc = op.fcre;
        kp = op.fpre;
    } else {
        kc = op.cre;
        kp = op.pre;
    }
    const R a = st ? -kp : kp, b = st ? -kc : kc;
    if constexpr (FU == 0) {
#pragma unroll
        for (int u = 0; u < kRegs; u++) {
            const R k = (__popc((uint32_t)u & op.gy) & 1) ? -b : b;
            const C2<R> v = x[u];
            x[u] = mk<R>(fma(-k, v.y, v.x), fma(k, v.x, v.y));
        }
    } else {
        constexpr int HB = 31 - __builtin_clz((unsigned)FU);
#pragma unroll
        for (int u0 = 0; u0 < kRegs; u0++) {
            if ((u0 >> HB) & 1) continue;
            const int u1 = u0 ^ FU;
            const bool neg = __popc((uint32_t)u0 & op.gy) & 1;
            const R k0 = neg ? -a : a, k1 = neg ? -b : b;
            const C2<R> x0 = x[u0], x1 = x[u1];
            if constexpr (IM) {
                x[u0] = mk<R>(fma(-k0, x1.y, x0.x), fma(k0, x1.x, x0.y));
                x[u1] = mk<R>(fma(-k1, x0.y, x1.x), fma(k1, x0.x, x1.y));
            } else {
                x[u0] = mk<R>(fma(k0, x1.x, x0.x), fma(k0, x1.y, x0.y));
                x[u1] = mk<R>(fma(k1, x0.x, x1.x), fma(k1, x0.y, x1.y));
            }
        }
    }
}

// The step's collected gadget factors, when no matrix of the step took them.
template <typename R>
__device__ __forceinline__ void reg_scale(C2<R> (&x)[kRegs], const ROp &op)
{
    R f;
    if constexpr (same_type<R, float>::value) f = op.fcs;
    else f = op.cs;
#pragma unroll
    for (int u = 0; u < kRegs; u++) x[u] = mk<R>(f * x[u].x, f * x[u].y);
}

// Dense gate on the FP32 matrix cores.  The wavefront's 64 lanes hold 16
// groups: lane L has member g = L / 16 of group L % 16 (g's bits are the lane
// coordinates), and for RM != 0 further members in registers u0 | rho.  Per
// register group one v_mfma_f32_16x16x4f32 K-step takes the real or the
// imaginary parts of one register; the output lands in the lane that holds
// the member (coefficients from mfma_coeffs).
//
// Coefficient layout: TW = 0, as the host writes them (each lane's NB * KS
// floats contiguous); TW > 0, the copy staged in LDS, in chunks of TW floats
// with the 64 lanes' chunks side by side, so that a wavefront reads 64
// consecutive chunks at once (no bank conflicts).
template <int RM, int TW = 0>
__device__ __forceinline__ void mfma_dense(float2 (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base,
                                           const float2 *__restrict__ mats)
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    constexpr int R = 1 << popcount_c(RM), KS = 2 * R, NB = R >= 2 ? R / 2 : 1;
    const float *A0 = reinterpret_cast<const float *>(mats + op.mat) + (threadIdx.x & 63u) * (TW ? TW : NB * KS);
    uint32_t tp = 0;
    for (int i = 0; i < op.nc; i++)
        tp |= (uint32_t)(((base >> op.cq[i]) ^ (uint64_t)__popc(tau & op.cm[i])) & 1ULL) << i;
    const uint32_t full = (1u << op.nc) - 1u;
#pragma unroll
    for (int u0 = 0; u0 < kRegs; u0++) {
        if (u0 & RM) continue;
        const bool ok = (tp ^ ((uint32_t)(op.qtab >> (4 * u0)) & 15u)) == full;
        if (op.nc && __ballot(ok) == 0) continue;   // controls off in the whole wavefront
        // coefficients for this register's lane-coordinate offset h(u0)
        const float *A = A0 + ((op.hsel >> (2 * u0)) & 3u) * (64 * NB * KS);
        float b[KS];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const float2 v = x[u0 | deposit_bits(r, RM)];
            b[2 * r] = v.x;
            b[2 * r + 1] = v.y;
        }
        // one output block (two registers' members) at a time
#pragma unroll
        for (int blk = 0; blk < NB; blk++) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; s++) {
                const int f = blk * KS + s;
                float a;
                if constexpr (TW == 4) {
                    // one 16-byte read per chunk (the LDS copy is 16-byte aligned)
                    const f32x4 v = *reinterpret_cast<const f32x4 *>(A + (f / 4) * 256);
                    a = v[f % 4];
                } else if constexpr (TW != 0) {
                    a = A[(f / (TW ? TW : 1)) * 64 * TW + f % (TW ? TW : 1)];
                } else {
                    a = A[f];
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[s], acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; i += 2) {
                const int r = (4 * blk + i) / 2;
                if (r < R && ok) x[u0 | deposit_bits(r, RM)] = make_float2(acc[i], acc[i + 1]);
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ void apply_reg_op(C2<R> (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base,
                                             const C2<R> *__restrict__ mats)
{
    constexpr bool f32 = same_type<R, float>::value;
    const C2<R> *m = mats + op.mat;
    // one switch (a jump table) over every operator code
    switch (op.code) {
    case 1: reg_dense<R, 1, false>(x, op, tau, base, m); break;
    case 2: reg_dense<R, 2, false>(x, op, tau, base, m); break;
    case 3: reg_dense<R, 3, false>(x, op, tau, base, m); break;
    case 4: reg_dense<R, 4, false>(x, op, tau, base, m); break;
    case 5: reg_dense<R, 5, false>(x, op, tau, base, m); break;
    case 6: reg_dense<R, 6, false>(x, op, tau, base, m); break;
    case 7: reg_dense<R, 7, false>(x, op, tau, base, m); break;
    case 8: reg_gadget<R, 0>(x, op, tau, base); break;
    case 9: reg_gadget<R, 1>(x, op, tau, base); break;
    case 10: reg_gadget<R, 2>(x, op, tau, base); break;
    case 11: reg_gadget<R, 3>(x, op, tau, base); break;
    case 12: reg_gadget<R, 4>(x, op, tau, base); break;
    case 13: reg_gadget<R, 5>(x, op, tau, base); break;
    case 14: reg_gadget<R, 6>(x, op, tau, base); break;
    case 15: reg_gadget<R, 7>(x, op, tau, base); break;
    case 16: reg_scale<R>(x, op); break;
    case 24: reg_gadget_f<R, 0, true>(x, op, tau, base); break;
    case 25: reg_gadget_f<R, 1, true>(x, op, tau, base); break;
    case 26: reg_gadget_f<R, 2, true>(x, op, tau, base); break;
    case 27: reg_gadget_f<R, 3, true>(x, op, tau, base); break;
    case 28: reg_gadget_f<R, 4, true>(x, op, tau, base); break;
    case 29: reg_gadget_f<R, 5, true>(x, op, tau, base); break;
    case 30: reg_gadget_f<R, 6, true>(x, op, tau, base); break;
    case 31: reg_gadget_f<R, 7, true>(x, op, tau, base); break;
    case 41: reg_gadget_f<R, 1, false>(x, op, tau, base); break;
    case 42: reg_gadget_f<R, 2, false>(x, op, tau, base); break;
    case 43: reg_gadget_f<R, 3, false>(x, op, tau, base); break;
    case 44: reg_gadget_f<R, 4, false>(x, op, tau, base); break;
    case 45: reg_gadget_f<R, 5, false>(x, op, tau, base); break;
    case 46: reg_gadget_f<R, 6, false>(x, op, tau, base); break;
    case 47: reg_gadget_f<R, 7, false>(x, op, tau, base); break;
    case 17: reg_dense<R, 1, true>(x, op, tau, base, m); break;
    case 18: reg_dense<R, 2, true>(x, op, tau, base, m); break;
    case 19: reg_dense<R, 3, true>(x, op, tau, base, m); break;
    case 20: reg_dense<R, 4, true>(x, op, tau, base, m); break;
    case 21: reg_dense<R, 5, true>(x, op, tau, base, m); break;
    case 22: reg_dense<R, 6, true>(x, op, tau, base, m); break;
    case 23: reg_dense<R, 7, true>(x, op, tau, base, m); break;
    case 32: if constexpr (f32) mfma_dense<0>(x, op, tau, base, mats); break;
    case 33: if constexpr (f32) mfma_dense<1>(x, op, tau, base, mats); break;
    case 34: if constexpr (f32) mfma_dense<2>(x, op, tau, base, mats); break;
    case 35: if constexpr (f32) mfma_dense<3>(x, op, tau, base, mats); break;
    case 36: if constexpr (f32) mfma_dense<4>(x, op, tau, base, mats); break;
    case 37: if constexpr (f32) mfma_dense<5>(x, op, tau, base, mats); break;
    case 38: if constexpr (f32) mfma_dense<6>(x, op, tau, base, mats); break;
    case 64 + 4 * 1: reg_sparse<R, 1, 0>(x, m); break;
    case 64 + 4 * 2: reg_sparse<R, 2, 0>(x, m); break;
    case 64 + 4 * 4: reg_sparse<R, 4, 0>(x, m); break;
    case 64 + 4 * 3: reg_sparse<R, 3, 0>(x, m); break;
    case 64 + 4 * 3 + 1: reg_sparse<R, 3, 1>(x, m); break;
    case 64 + 4 * 3 + 2: reg_sparse<R, 3, 2>(x, m); break;
    case 64 + 4 * 3 + 3: reg_sparse<R, 3, 3>(x, m); break;
    case 64 + 4 * 5: reg_sparse<R, 5, 0>(x, m); break;
    case 64 + 4 * 5 + 1: reg_sparse<R, 5, 1>(x, m); break;
    case 64 + 4 * 5 + 2: reg_sparse<R, 5, 2>(x, m); break;
    case 64 + 4 * 5 + 3: reg_sparse<R, 5, 3>(x, m); break;
    case 64 + 4 * 6: reg_sparse<R, 6, 0>(x, m); break;
    case 64 + 4 * 6 + 1: reg_sparse<R, 6, 1>(x, m); break;
    case 64 + 4 * 6 + 2: reg_sparse<R, 6, 2>(x, m); break;
    case 64 + 4 * 6 + 3: reg_sparse<R, 6, 3>(x, m); break;
    default: break;
    }
}


// Moves the tile from phase Q's register layout to phase P's through LDS and
// returns P's tau of this thread (tau_q: Q's).
template <typename R>
__device__ __forceinline__ uint32_t tile_exchange(C2<R> (&x)[kRegs], unsigned char *lds, uint32_t tau_q,
                                                  const RPhase &Q, const RPhase &P)
{
    constexpr int sh = sizeof(C2<R>) == 8 ? 3 : 4;
    const uint32_t tn = tau_of(threadIdx.x, P);
    const uint32_t ob = tau_q << sh, nb = tn << sh;
    __syncthreads();   // earlier reads of the LDS tile are done
#pragma unroll
    for (int u = 0; u < kRegs; u++) *(C2<R> *)(lds + (ob ^ (Q.rho[u] << sh))) = x[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kRegs; u++) x[u] = *(const C2<R> *)(lds + (nb ^ (P.rho[u] << sh)));
    return tn;
}

// Blocks of 2^(d - kRegBits) threads, each walking a run of tiles: with
// `chunk` set, block b takes the consecutive tiles b per .. b per + per - 1
// (per = ceil(num_tiles / gridDim.x)); otherwise tiles b + k gridDim.x.  The
// consecutive runs measured up to 1.6x faster than the strided walk for
// tiles that hold a high qubit (the strided walk's blocks drift apart across
// the state), and no slower otherwise.  A tile is read from HBM straight into
// the first phase's layout and written from the last one's; the next tile's
// loads are issued before the current tile's operators run (phases(x, base):
// every phase of the step), so they are in flight during the arithmetic
// (barriers wait for LDS only).  Tiles are disjoint, so the early read sees no
// write of this launch.
template <typename R, typename Phases>
__device__ __forceinline__ void tile_walk(C2<R> *__restrict__ a, uint64_t num_tiles, const InsertPlan &plan,
                                          const RPhase &first, const RPhase &last, int lb, bool chunk,
                                          Phases phases)
{
    const uint32_t t = threadIdx.x;
    const uint64_t xg = thread_offset(t, lb, first);
    const uint64_t xs = thread_offset(t, lb, last);
    const uint64_t per = chunk ? (num_tiles + gridDim.x - 1) / gridDim.x : 1;
    const uint64_t step = chunk ? 1 : gridDim.x;
    uint64_t tile = (uint64_t)blockIdx.x * per;
    uint64_t end = chunk ? tile + per : num_tiles;
    if (end > num_tiles) end = num_tiles;
    if (tile >= end) return;
    C2<R> x[kRegs];
    {
        const uint64_t b0 = insert_zeros(tile, plan);
#pragma unroll
        for (int u = 0; u < kRegs; u++) x[u] = a[b0 ^ xg ^ first.yaddr[u]];
        // the first tile is waited for here, so that inside the loop the
        // only memory wait is for the prefetch, never for earlier stores
#pragma unroll
        for (int u = 0; u < kRegs; u++) asm volatile("" ::"v"(x[u].x), "v"(x[u].y));
    }
    for (; tile < end; tile += step) {
        const uint64_t base = insert_zeros(tile, plan);
        const uint64_t next = tile + step;
        const bool more = next < end;
        // defined on every path (zeros after the last tile): registers that
        // are undefined on one path of the loop have been given to other
        // values by the compiler's register allocation
        C2<R> nx[kRegs];
#pragma unroll
        for (int u = 0; u < kRegs; u++) nx[u] = mk<R>(R(0), R(0));
        if (more) {
            const uint64_t nb = insert_zeros(next, plan);
#pragma unroll
            for (int u = 0; u < kRegs; u++) nx[u] = a[nb ^ xg ^ first.yaddr[u]];
        }
        phases(x, base);
#pragma unroll
        for (int u = 0; u < kRegs; u++) a[base ^ xs ^ last.yaddr[u]] = x[u];
#pragma unroll
        for (int u = 0; u < kRegs; u++) x[u] = nx[u];
    }
}

}  // namespace qs
