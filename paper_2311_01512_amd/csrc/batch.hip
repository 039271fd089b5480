// Batched execution of many parametrised circuits of uneven size, with
// per-circuit Pauli-sum energies and adjoint-method gradients.
//
// Each circuit is split into steps: a step owns a set Q of at most T qubits
// (always including the lowest C qubits, so tiles are read in runs of 2^C
// consecutive amplitudes) and the operators that act inside Q or are
// diagonal.  A step streams the state through LDS one 2^|Q| tile at a time
// (the tile number is spread over the qubits outside Q) and applies its
// operators to the tile.  Operators are absorbed into a step only if they
// commute with every operator left behind (no shared qubit), so the order of
// the circuit is respected.  All circuits' s-th steps form one kernel launch.
#include "batch_dev.hpp"
#include "circuit.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <sstream>
#include <string>

namespace qs {

struct BOp {
    int kind, q0, q1, pauli, param;
    double scale;
    cd m[4];
    int logical = 1;  // operators of the recorded circuit it stands for (0: part of a decomposed gadget)
    uint64_t support() const { return (1ULL << q0) | (kind == BOP_CZ ? (1ULL << q1) : 0ULL); }
};

struct BStep {
    uint64_t qmask;
    std::vector<int> ops;
};

struct BCirc {
    int n, num_params;
    std::vector<BOp> ops;
    std::vector<int> codes;
    std::vector<double> coeffs;
    std::vector<BStep> steps;
    uint64_t amp_off;
    int param_off;
};

struct DTerm {
    uint64_t x, yz;
    double cre, cim;  // h_n i^{#Y}
};

// (re, im) summed over the block; valid in thread 0.
__device__ void bblock_sum2(double &re, double &im, double *scratch)
{
    re = bwave_sum(re);
    im = bwave_sum(im);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        scratch[2 * wave] = re;
        scratch[2 * wave + 1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
            a += scratch[2 * w];
            b += scratch[2 * w + 1];
        }
        re = a;
        im = b;
    }
}

__device__ __forceinline__ uint64_t tile_offset(int j, const DStep &st)
{
    uint64_t o = 0;
    for (int b = 0; b < st.qn; b++) o |= (uint64_t)((j >> b) & 1) << st.qpos[b];
    return o;
}

// cos and sin of every rotation's angle scale * parameter, once per run.
__global__ __launch_bounds__(256) void k_batch_trig(const DOp *__restrict__ ops, int num_ops,
                                                     const double *__restrict__ params, double *__restrict__ trig)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= num_ops) return;
    const DOp op = ops[k];
    double s = 0.0, c = 1.0;
    if (op.kind == BOP_ROT) sincos(op.scale * params[op.param], &s, &c);
    trig[2 * k] = c;
    trig[2 * k + 1] = s;
}

template <typename R>
__device__ void tile_gate(C2<R> *v, int qn, int pos, const C2<R> (&u)[4])
{
    const int np = 1 << (qn - 1);
    const int lo = (1 << pos) - 1;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int j0 = (p & lo) | ((p & ~lo) << 1), j1 = j0 | (1 << pos);
        const C2<R> a = v[j0], b = v[j1];
        C2<R> x = mk<R>(0, 0), y = mk<R>(0, 0);
        cmac<R>(x, u[0], a);
        cmac<R>(x, u[1], b);
        cmac<R>(y, u[2], a);
        cmac<R>(y, u[3], b);
        v[j0] = x;
        v[j1] = y;
    }
}

template <typename R>
__device__ void tile_cz(C2<R> *v, int qn, const DOp &op, uint64_t base)
{
    const int T = 1 << qn;
    const int b0 = op.pos0 < 0 ? (int)((base >> op.q0) & 1) : -1;
    const int b1 = op.pos1 < 0 ? (int)((base >> op.q1) & 1) : -1;
    if (b0 == 0 || b1 == 0) return;   // the tile lies where a control bit is 0
    for (int j = threadIdx.x; j < T; j += blockDim.x) {
        const int x0 = b0 < 0 ? (j >> op.pos0) & 1 : 1;
        const int x1 = b1 < 0 ? (j >> op.pos1) & 1 : 1;
        if (x0 & x1) v[j] = mk<R>(-v[j].x, -v[j].y);
    }
}

template <typename R>
__device__ void tile_apply(C2<R> *v, int qn, const DOp &op, uint64_t base, const double *trig, int dir)
{
    if (op.kind == BOP_CZ) {
        tile_cz<R>(v, qn, op, base);
    } else {
        C2<R> u[4];
        op_matrix<R>(op, trig, dir, u);
        tile_gate<R>(v, qn, op.pos0, u);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_batch_forward(C2<R> *__restrict__ amps, const DStep *__restrict__ steps,
                                                        const DOp *__restrict__ ops, const uint2 *__restrict__ work,
                                                        const double *__restrict__ trig)
{
    extern __shared__ unsigned char lds_raw[];
    C2<R> *v = reinterpret_cast<C2<R> *>(lds_raw);
    const uint2 w = work[blockIdx.x];
    const DStep &st = steps[w.x];
    const uint64_t base = insert_zeros(w.y, st.plan);
    C2<R> *a = amps + st.amp_off;
    const int T = 1 << st.qn;
    for (int j = threadIdx.x; j < T; j += blockDim.x) v[j] = load_amp<R>(a, base | tile_offset(j, st), st.first);
    __syncthreads();
    for (int k = st.op_begin; k < st.op_end; k++) {
        tile_apply<R>(v, st.qn, ops[k], base, trig + 2 * k, +1);
        __syncthreads();
    }
    for (int j = threadIdx.x; j < T; j += blockDim.x) a[base | tile_offset(j, st)] = v[j];
}

// Adjoint sweep over one tile of phi and lambda: for each operator, last
// first, the rotation's partial Im <lambda|P|phi> over the tile (the
// gradient -2 s Im <lambda|P|phi> needs no real part), then
// phi <- U^dagger phi and lambda <- U^dagger lambda.  For a rotation both
// happen in one pass over the pairs (j0, j1) it couples; each wavefront
// reduces its share in FP64 and leaves it in LDS, and thread 0 adds the
// wavefronts' shares (fixed order) after the barrier that ends the operator,
// so a rotation costs no barrier of its own.
template <typename R>
__global__ __launch_bounds__(256) void k_batch_backward(C2<R> *__restrict__ amps, uint64_t lambda_base,
                                                         const DStep *__restrict__ steps, const DOp *__restrict__ ops,
                                                         const uint2 *__restrict__ work,
                                                         const double *__restrict__ trig, double *__restrict__ gpart)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[2][4];   // two rotations in flight, Im of up to 4 wavefronts
    const uint2 w = work[blockIdx.x];
    const DStep &st = steps[w.x];
    const int T = 1 << st.qn;
    C2<R> *phi = reinterpret_cast<C2<R> *>(lds_raw);
    C2<R> *lam = phi + T;
    const uint64_t base = insert_zeros(w.y, st.plan);
    C2<R> *a = amps + st.amp_off;
    C2<R> *l = amps + lambda_base + st.amp_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int j = threadIdx.x; j < T; j += blockDim.x) {
        const uint64_t o = base | tile_offset(j, st);
        phi[j] = a[o];
        lam[j] = l[o];
    }
    __syncthreads();
    uint64_t pend = ~0ULL;   // partial index of the rotation whose wave sums sit in red[pslot]
    int pslot = 0;
    auto flush = [&]() {
        if (pend != ~0ULL && threadIdx.x == 0) {
            double im = 0.0;
            for (int v = 0; v < nwaves; v++) im += red[pslot][v];
            gpart[pend] = im;
        }
        pend = ~0ULL;
    };
    for (int k = st.op_end - 1; k >= st.op_begin; k--) {
        const DOp &op = ops[k];
        flush();   // the previous operator's barrier made its wave sums visible
        if (op.kind == BOP_CZ) {
            tile_cz<R>(phi, st.qn, op, base);
            tile_cz<R>(lam, st.qn, op, base);
        } else {
            C2<R> u[4];
            op_matrix<R>(op, trig + 2 * k, -1, u);
            if (op.grad < 0) {
                tile_gate<R>(phi, st.qn, op.pos0, u);
                tile_gate<R>(lam, st.qn, op.pos0, u);
            } else {
                const int pos = op.pos0, lo = (1 << pos) - 1, np = T >> 1;
                double im = 0.0;
                for (int p = threadIdx.x; p < np; p += blockDim.x) {
                    const int j0 = (p & lo) | ((p & ~lo) << 1), j1 = j0 | (1 << pos);
                    const C2<R> f0 = phi[j0], f1 = phi[j1], y0 = lam[j0], y1 = lam[j1];
                    C2<R> p0, p1;   // (P phi) at j0 and j1
                    if (op.pauli == 1) {
                        p0 = f1;
                        p1 = f0;
                    } else if (op.pauli == 2) {   // Y: -i phi_j1 at j0, +i phi_j0 at j1
                        p0 = mk<R>(f1.y, -f1.x);
                        p1 = mk<R>(-f0.y, f0.x);
                    } else {
                        p0 = f0;
                        p1 = mk<R>(-f1.x, -f1.y);
                    }
                    im += (double)y0.x * p0.y - (double)y0.y * p0.x + (double)y1.x * p1.y - (double)y1.y * p1.x;
                    C2<R> g0 = mk<R>(0, 0), g1 = mk<R>(0, 0), h0 = mk<R>(0, 0), h1 = mk<R>(0, 0);
                    cmac<R>(g0, u[0], f0);
                    cmac<R>(g0, u[1], f1);
                    cmac<R>(g1, u[2], f0);
                    cmac<R>(g1, u[3], f1);
                    cmac<R>(h0, u[0], y0);
                    cmac<R>(h0, u[1], y1);
                    cmac<R>(h1, u[2], y0);
                    cmac<R>(h1, u[3], y1);
                    phi[j0] = g0;
                    phi[j1] = g1;
                    lam[j0] = h0;
                    lam[j1] = h1;
                }
                im = bwave_sum(im);
                pslot = k & 1;
                if (lane == 0) red[pslot][wave] = im;
                pend = op.gpart + w.y;
            }
        }
        __syncthreads();
    }
    flush();
    for (int j = threadIdx.x; j < T; j += blockDim.x) {
        const uint64_t o = base | tile_offset(j, st);
        a[o] = phi[j];
        l[o] = lam[j];
    }
}

// ---- register-phase path (tiles of >= 2^kRegMinQubits amplitudes) ----------------------

template <typename R>
__global__ __launch_bounds__(512) void k_batch_forward_reg(C2<R> *__restrict__ amps, const DStep *__restrict__ steps,
                                                            const BPhase *__restrict__ phases,
                                                            const DOp *__restrict__ ops, const uint2 *__restrict__ work,
                                                            const double *__restrict__ trig)
{
    extern __shared__ unsigned char lds_raw[];
    C2<R> *v = reinterpret_cast<C2<R> *>(lds_raw);
    const uint2 w = work[blockIdx.x];
    const DStep &st = steps[w.x];
    const uint64_t base = insert_zeros(w.y, st.plan);
    C2<R> *a = amps + st.amp_off;
    const uint32_t t = threadIdx.x;
    const bool active = t < (1u << (st.qn - 3));   // whole wavefronts (qn >= 9)
    const BPhase &f = phases[st.ph_begin];
    uint32_t tau = bphase_tau(t, f);
    C2<R> x[8];
    if (active) {
        const uint64_t xo = base | tile_offset_bits(tau, st);
        const RegOffsets ro(f, st);
#pragma unroll
        for (int u = 0; u < 8; u++) x[u] = load_amp<R>(a, xo | ro(u), st.first);
    }
    for (int p = st.ph_begin; p < st.ph_end; p++) {
        const BPhase &P = phases[p];
        if (p > st.ph_begin) tau = bphase_exchange<R>(x, v, tau, phases[p - 1], P, active);
        if (!active) continue;
        uint32_t czm = 0;   // sign mask of the current run of CZs
        for (int k = P.op_begin; k < P.op_end; k++) fwd_op<R>(x, ops[k], k, trig, tau, base, czm);
    }
    if (active) {
        const uint64_t xo = base | tile_offset_bits(tau, st);
        const RegOffsets ro(phases[st.ph_end - 1], st);
#pragma unroll
        for (int u = 0; u < 8; u++) a[xo | ro(u)] = x[u];
    }
}

// Adjoint sweep on registers: phases and operators last first; a rotation's
// partial Im <lambda|P|phi> comes from the register pairs it couples, before
// U^dagger is applied to both states.  Each row of 16 lanes leaves its
// partial in the rotation's LDS slots; after the barrier that opens the next
// exchange one thread per rotation adds the rows' partials (fixed order),
// and those reads complete before the exchange's second barrier, after
// which the next phase writes the slots again.
template <typename R>
__global__ __launch_bounds__(512) void k_batch_backward_reg(C2<R> *__restrict__ amps, uint64_t lambda_base,
                                                             const DStep *__restrict__ steps,
                                                             const BPhase *__restrict__ phases,
                                                             const DOp *__restrict__ ops,
                                                             const uint2 *__restrict__ work,
                                                             const double *__restrict__ trig,
                                                             double *__restrict__ gpart)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[kPhaseRotMax][kRedRows];
    const uint2 w = work[blockIdx.x];
    const DStep &st = steps[w.x];
    const uint64_t base = insert_zeros(w.y, st.plan);
    const int T = 1 << st.qn;
    C2<R> *vphi = reinterpret_cast<C2<R> *>(lds_raw);
    C2<R> *vlam = vphi + T;
    C2<R> *a = amps + st.amp_off;
    C2<R> *l = amps + lambda_base + st.amp_off;
    const uint32_t t = threadIdx.x;
    const uint32_t nthr = 1u << (st.qn - 3);
    const bool active = t < nthr;
    const int lane = t & 63, wave = t >> 6, nwaves = (int)(nthr >> 6);
    const BPhase &f = phases[st.ph_end - 1];
    uint32_t tau = bphase_tau(t, f);
    C2<R> x[8], y[8];
    if (active) {
        const uint64_t xo = base | tile_offset_bits(tau, st);
        const RegOffsets ro(f, st);
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint64_t o = xo | ro(u);
            x[u] = a[o];
            y[u] = l[o];
        }
    }
    for (int p = st.ph_end - 1; p >= st.ph_begin; p--) {
        const BPhase &P = phases[p];
        if (p < st.ph_end - 1) {
            const BPhase &D = phases[p + 1];   // the finished phase
            __syncthreads();   // earlier LDS reads done; the finished phase's partials visible
            flush_phase(ops, D.op_begin, D.op_end, red, nwaves, w.y, gpart);
            tau = bphase_exchange2<R>(x, y, vphi, vlam, tau, D, P, active);
        }
        if (!active) continue;
        uint32_t czm = 0;   // sign mask of the current run of CZs
        for (int k = P.op_end - 1; k >= P.op_begin; k--) bwd_op<R>(x, y, ops[k], k, trig, tau, base, czm, red, lane, wave);
    }
    __syncthreads();
    flush_phase(ops, phases[st.ph_begin].op_begin, phases[st.ph_begin].op_end, red, nwaves, w.y, gpart);
    if (active) {
        const uint64_t xo = base | tile_offset_bits(tau, st);
        const RegOffsets ro(phases[st.ph_begin], st);
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint64_t o = xo | ro(u);
            a[o] = x[u];
            l[o] = y[u];
        }
    }
}

// Per-block circuit table of the flat amplitude range.
struct BlockMap {
    const int *circ;         // circuit of each 256-amplitude block
    const uint64_t *start;   // first local index of each block
};

// |0..0> in the listed 256-amplitude blocks.
template <typename R>
__global__ __launch_bounds__(256) void k_batch_init(C2<R> *__restrict__ amps, BlockMap bm, const int *__restrict__ blocks,
                                                     const uint64_t *__restrict__ offs, const int *__restrict__ nq)
{
    const int blk = blocks[blockIdx.x];
    const int c = bm.circ[blk];
    const uint64_t i = bm.start[blk] + threadIdx.x;
    if (i < (1ULL << nq[c])) amps[offs[c] + i] = mk<R>(i == 0 ? R(1) : R(0), R(0));
}

constexpr int kTermGroup = 4;   // Hamiltonian terms gathered together

// lambda = H phi with (P phi)_i = beta_{i^x} phi_{i^x}, beta_y = i^{#Y} (-1)^{popc(y & yz)};
// energy partial sum_i conj(phi_i) lambda_i per block.
template <typename R>
__global__ __launch_bounds__(256) void k_batch_hamiltonian(C2<R> *__restrict__ amps, uint64_t lambda_base, BlockMap bm,
                                                            const uint64_t *__restrict__ offs,
                                                            const int *__restrict__ nq, const int *__restrict__ term_off,
                                                            const DTerm *__restrict__ terms, double *__restrict__ epart)
{
    __shared__ double red[32];
    const int c = bm.circ[blockIdx.x];
    const uint64_t i = bm.start[blockIdx.x] + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (i < (1ULL << nq[c])) {
        const C2<R> *phi = amps + offs[c];
        double lr = 0.0, li = 0.0;
        const int tb = term_off[c], te = term_off[c + 1];
        // indices within a circuit of at most 30 qubits: 32-bit
        const uint32_t i32 = (uint32_t)i;
        // a group's gathers in flight before their sums (same order of
        // additions as one term at a time; the host pads every circuit's
        // terms to whole groups with zero terms)
        constexpr int G = kTermGroup;
        for (int t0 = tb; t0 < te; t0 += G) {
            C2<R> xs[G];
#pragma unroll
            for (int u = 0; u < G; u++) xs[u] = phi[i32 ^ (uint32_t)terms[t0 + u].x];
#pragma unroll
            for (int u = 0; u < G; u++) {
                const DTerm tm = terms[t0 + u];
                const uint32_t j = i32 ^ (uint32_t)tm.x;
                const double s = (__popc(j & (uint32_t)tm.yz) & 1) ? -1.0 : 1.0;
                const C2<R> x = xs[u];
                lr += s * (tm.cre * x.x - tm.cim * x.y);
                li += s * (tm.cre * x.y + tm.cim * x.x);
            }
        }
        amps[lambda_base + offs[c] + i] = mk<R>((R)lr, (R)li);
        const C2<R> p = phi[i];
        re = (double)p.x * lr + (double)p.y * li;
        im = (double)p.x * li - (double)p.y * lr;
    }
    bblock_sum2(re, im, red);
    if (threadIdx.x == 0) {
        epart[2 * blockIdx.x] = re;
        epart[2 * blockIdx.x + 1] = im;
    }
}

// One block per circuit: fixed-order sum of its blocks' energy partials.
__global__ __launch_bounds__(256) void k_batch_energy(const double *__restrict__ epart, const int *__restrict__ first_block,
                                                       double *__restrict__ energy)
{
    __shared__ double red[32];
    const int c = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int b = first_block[c] + threadIdx.x; b < first_block[c + 1]; b += blockDim.x) {
        re += epart[2 * b];
        im += epart[2 * b + 1];
    }
    bblock_sum2(re, im, red);
    if (threadIdx.x == 0) {
        energy[2 * c] = re;
        energy[2 * c + 1] = im;
    }
}

// One thread per rotation: fixed-order sum over its tiles.
__global__ __launch_bounds__(256) void k_batch_grad(const double *__restrict__ gpart, const uint64_t *__restrict__ first,
                                                     int num_rot, double *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= num_rot) return;
    double im = 0.0;
    for (uint64_t t = first[r]; t < first[r + 1]; t++) im += gpart[t];
    out[r] = im;
}

}  // namespace qs

using namespace qs;

struct qs_batch {
    int precision;
    std::vector<BCirc> circs;
    bool compiled = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int use_graph = 1;
    int tile_qubits = 12, low_qubits = 3;
    // device
    void *amps = nullptr;
    uint64_t total_amps = 0;     // per region (phi); lambda follows
    DStep *d_steps = nullptr;
    DOp *d_ops = nullptr;
    std::vector<uint2 *> d_work;          // per phase
    std::vector<unsigned> phase_blocks;
    int *d_bm_circ = nullptr;
    uint64_t *d_bm_start = nullptr;
    unsigned amp_blocks = 0;
    int *d_init_blocks = nullptr;   // 256-amplitude blocks of the circuits without steps
    unsigned init_blocks = 0;
    uint64_t *d_offs = nullptr;
    int *d_nq = nullptr;
    int *d_term_off = nullptr;
    DTerm *d_terms = nullptr;
    int *d_first_block = nullptr;
    double *d_epart = nullptr, *d_energy = nullptr, *h_energy = nullptr;
    double *d_gpart = nullptr, *d_gop = nullptr, *h_gop = nullptr;
    uint64_t *d_gfirst = nullptr;
    int num_rot = 0;
    std::vector<int> rot_param;      // global parameter of each rotation slot
    std::vector<double> rot_scale;
    double *d_params = nullptr, *h_params = nullptr;
    double *d_trig = nullptr;   // cos, sin of every operator's angle
    std::vector<uint2 *> d_work_reg;          // register-path work lists per launch step
    std::vector<unsigned> phase_blocks_reg;
    BPhase *d_phases = nullptr;
    int num_ops = 0;
    int total_params = 0;
    hipGraphExec_t g_fwd = nullptr, g_full = nullptr;
    hipGraph_t gr_fwd = nullptr, gr_full = nullptr;
    bool last_run_had_grads = false;
    // host copies of the device tables, for run-time specialisation
    std::vector<DStep> h_steps;
    std::vector<DOp> h_ops;
    std::vector<BPhase> h_phases;
    std::vector<int> step_launch;    // launch index (step s of its circuit) of every step
    // specialised register-path kernels per launch index (null: the generic ones)
    std::vector<void *> jit_modules;
    std::vector<void *> jit_fwd, jit_bwd;
    int num_programs = 0;
};

namespace qs {

static void plan_circuit(BCirc &c, int TQ, int C)
{
    const int L = (int)c.ops.size();
    std::vector<char> placed(L, 0);
    int remaining = L;
    const uint64_t all = (c.n >= 64) ? ~0ULL : ((1ULL << c.n) - 1ULL);
    c.steps.clear();
    while (remaining > 0) {
        uint64_t Q = 0;
        if (c.n <= TQ) {
            Q = all;
        } else {
            for (int b = 0; b < C; b++) Q |= 1ULL << b;
            uint64_t blocked = 0;
            for (int k = 0; k < L && __builtin_popcountll(Q) < TQ; k++) {
                if (placed[k]) continue;
                const uint64_t s = c.ops[k].support();
                if (s & blocked) {
                    blocked |= s;
                    continue;
                }
                if (c.ops[k].kind == BOP_CZ) continue;   // diagonal: needs no tile qubit
                Q |= s;
            }
            // fill the step to TQ qubits with the lowest free ones (longer
            // contiguous runs, and tiles the register path takes)
            for (int q = C; q < c.n && __builtin_popcountll(Q) < TQ; q++) Q |= 1ULL << q;
        }
        BStep st;
        st.qmask = Q;
        uint64_t blocked = 0;
        for (int k = 0; k < L; k++) {
            if (placed[k]) continue;
            const BOp &op = c.ops[k];
            const uint64_t s = op.support();
            if (s & blocked) {
                blocked |= s;
                continue;
            }
            if (op.kind == BOP_CZ || (s & ~Q) == 0) {
                st.ops.push_back(k);
                placed[k] = 1;
                remaining--;
            } else {
                blocked |= s;
            }
        }
        c.steps.push_back(std::move(st));
    }
}

static int launch_phase_kernels(qs_batch *b, bool grads)
{
    const size_t ab = b->precision == QS_C64 ? 8 : 16;
    const size_t lds1 = ((size_t)1 << b->tile_qubits) * ab;
    const int P = (int)b->d_work.size();
    hipLaunchKernelGGL(k_batch_trig, dim3((unsigned)((b->num_ops + 255) / 256)), dim3(256), 0, b->stream,
                       (const DOp *)b->d_ops, b->num_ops, (const double *)b->d_params, b->d_trig);
    QS_LAUNCH_CHECK();
    // |0..0> for circuits without operators (a circuit's first step reads
    // |0..0> itself)
    if (b->init_blocks > 0) {
        if (b->precision == QS_C64)
            hipLaunchKernelGGL(k_batch_init<float>, dim3(b->init_blocks), dim3(256), 0, b->stream, (float2 *)b->amps,
                               BlockMap{b->d_bm_circ, b->d_bm_start}, (const int *)b->d_init_blocks,
                               (const uint64_t *)b->d_offs, (const int *)b->d_nq);
        else
            hipLaunchKernelGGL(k_batch_init<double>, dim3(b->init_blocks), dim3(256), 0, b->stream,
                               (double2 *)b->amps, BlockMap{b->d_bm_circ, b->d_bm_start}, (const int *)b->d_init_blocks,
                               (const uint64_t *)b->d_offs, (const int *)b->d_nq);
        QS_LAUNCH_CHECK();
    }
    const unsigned rblock = 1u << (b->tile_qubits - 3);   // register path: 8 amplitudes per thread
    for (int p = 0; p < P; p++) {
        if (b->phase_blocks[p] > 0) {
            if (b->precision == QS_C64)
                hipLaunchKernelGGL(k_batch_forward<float>, dim3(b->phase_blocks[p]), dim3(256), lds1, b->stream,
                                   (float2 *)b->amps, (const DStep *)b->d_steps, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work[p], (const double *)b->d_trig);
            else
                hipLaunchKernelGGL(k_batch_forward<double>, dim3(b->phase_blocks[p]), dim3(256), lds1, b->stream,
                                   (double2 *)b->amps, (const DStep *)b->d_steps, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work[p], (const double *)b->d_trig);
            QS_LAUNCH_CHECK();
        }
        if (b->phase_blocks_reg[p] > 0 && p < (int)b->jit_fwd.size() && b->jit_fwd[p]) {
            void *amps = b->amps;
            const void *steps = b->d_steps, *work = b->d_work_reg[p], *trig = b->d_trig;
            void *args[] = {&amps, &steps, &work, &trig};
            QS_HIP(hipModuleLaunchKernel((hipFunction_t)b->jit_fwd[p], b->phase_blocks_reg[p], 1, 1, rblock, 1, 1,
                                         (unsigned)lds1, b->stream, args, nullptr));
        } else if (b->phase_blocks_reg[p] > 0) {
            if (b->precision == QS_C64)
                hipLaunchKernelGGL(k_batch_forward_reg<float>, dim3(b->phase_blocks_reg[p]), dim3(rblock), lds1,
                                   b->stream, (float2 *)b->amps, (const DStep *)b->d_steps,
                                   (const BPhase *)b->d_phases, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work_reg[p], (const double *)b->d_trig);
            else
                hipLaunchKernelGGL(k_batch_forward_reg<double>, dim3(b->phase_blocks_reg[p]), dim3(rblock), lds1,
                                   b->stream, (double2 *)b->amps, (const DStep *)b->d_steps,
                                   (const BPhase *)b->d_phases, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work_reg[p], (const double *)b->d_trig);
            QS_LAUNCH_CHECK();
        }
    }
    const BlockMap bm{b->d_bm_circ, b->d_bm_start};
    if (b->precision == QS_C64)
        hipLaunchKernelGGL(k_batch_hamiltonian<float>, dim3(b->amp_blocks), dim3(256), 0, b->stream, (float2 *)b->amps,
                           b->total_amps, bm, (const uint64_t *)b->d_offs, (const int *)b->d_nq,
                           (const int *)b->d_term_off, (const DTerm *)b->d_terms, b->d_epart);
    else
        hipLaunchKernelGGL(k_batch_hamiltonian<double>, dim3(b->amp_blocks), dim3(256), 0, b->stream,
                           (double2 *)b->amps, b->total_amps, bm, (const uint64_t *)b->d_offs, (const int *)b->d_nq,
                           (const int *)b->d_term_off, (const DTerm *)b->d_terms, b->d_epart);
    QS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_batch_energy, dim3((unsigned)b->circs.size()), dim3(256), 0, b->stream,
                       (const double *)b->d_epart, (const int *)b->d_first_block, b->d_energy);
    QS_LAUNCH_CHECK();
    if (!grads) return QS_OK;
    for (int p = P - 1; p >= 0; p--) {
        if (b->phase_blocks[p] > 0) {
            if (b->precision == QS_C64)
                hipLaunchKernelGGL(k_batch_backward<float>, dim3(b->phase_blocks[p]), dim3(256), 2 * lds1,
                                   b->stream, (float2 *)b->amps, b->total_amps, (const DStep *)b->d_steps,
                                   (const DOp *)b->d_ops, (const uint2 *)b->d_work[p], (const double *)b->d_trig,
                                   b->d_gpart);
            else
                hipLaunchKernelGGL(k_batch_backward<double>, dim3(b->phase_blocks[p]), dim3(256), 2 * lds1,
                                   b->stream, (double2 *)b->amps, b->total_amps, (const DStep *)b->d_steps,
                                   (const DOp *)b->d_ops, (const uint2 *)b->d_work[p], (const double *)b->d_trig,
                                   b->d_gpart);
            QS_LAUNCH_CHECK();
        }
        if (b->phase_blocks_reg[p] > 0 && p < (int)b->jit_bwd.size() && b->jit_bwd[p]) {
            void *amps = b->amps, *gpart = b->d_gpart;
            unsigned long long lambda_base = b->total_amps;
            const void *steps = b->d_steps, *ops = b->d_ops, *work = b->d_work_reg[p], *trig = b->d_trig;
            void *args[] = {&amps, &lambda_base, &steps, &ops, &work, &trig, &gpart};
            QS_HIP(hipModuleLaunchKernel((hipFunction_t)b->jit_bwd[p], b->phase_blocks_reg[p], 1, 1, rblock, 1, 1,
                                         (unsigned)(2 * lds1), b->stream, args, nullptr));
        } else if (b->phase_blocks_reg[p] > 0) {
            if (b->precision == QS_C64)
                hipLaunchKernelGGL(k_batch_backward_reg<float>, dim3(b->phase_blocks_reg[p]), dim3(rblock),
                                   2 * lds1, b->stream, (float2 *)b->amps, b->total_amps,
                                   (const DStep *)b->d_steps, (const BPhase *)b->d_phases, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work_reg[p], (const double *)b->d_trig, b->d_gpart);
            else
                hipLaunchKernelGGL(k_batch_backward_reg<double>, dim3(b->phase_blocks_reg[p]), dim3(rblock),
                                   2 * lds1, b->stream, (double2 *)b->amps, b->total_amps,
                                   (const DStep *)b->d_steps, (const BPhase *)b->d_phases, (const DOp *)b->d_ops,
                                   (const uint2 *)b->d_work_reg[p], (const double *)b->d_trig, b->d_gpart);
            QS_LAUNCH_CHECK();
        }
    }
    if (b->num_rot > 0) {
        hipLaunchKernelGGL(k_batch_grad, dim3((b->num_rot + 255) / 256), dim3(256), 0, b->stream,
                           (const double *)b->d_gpart, (const uint64_t *)b->d_gfirst, b->num_rot, b->d_gop);
        QS_LAUNCH_CHECK();
    }
    return QS_OK;
}

static int capture(qs_batch *b, bool grads, hipGraph_t *g, hipGraphExec_t *ge)
{
    QS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_phase_kernels(b, grads);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (rc != QS_OK) return rc;
    if (e != hipSuccess) return fail(QS_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    QS_HIP(hipGraphInstantiate(ge, graph, nullptr, nullptr, 0));
    *g = graph;
    return QS_OK;
}

template <typename P>
static int upload(P **dst, const void *src, size_t bytes)
{
    if (hipMalloc((void **)dst, bytes > 0 ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(QS_E_ALLOC, "device allocation failed");
    }
    if (src && bytes > 0) QS_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return QS_OK;
}

// Unloads the specialised step kernels (the caller has waited for the
// batch's stream).
static void release_jit(qs_batch *b)
{
    for (void *m : b->jit_modules) (void)hipModuleUnload((hipModule_t)m);
    b->jit_modules.clear();
    b->jit_fwd.clear();
    b->jit_bwd.clear();
    b->num_programs = 0;
}

static void release(qs_batch *b)
{
    auto f = [](void *p) {
        if (p) (void)hipFree(p);
    };
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->own_stream = false;
    b->stream = nullptr;
    if (b->g_fwd) (void)hipGraphExecDestroy(b->g_fwd);
    if (b->g_full) (void)hipGraphExecDestroy(b->g_full);
    if (b->gr_fwd) (void)hipGraphDestroy(b->gr_fwd);
    if (b->gr_full) (void)hipGraphDestroy(b->gr_full);
    b->g_fwd = b->g_full = nullptr;
    b->gr_fwd = b->gr_full = nullptr;
    release_jit(b);   // after the graphs that launch its kernels
    f(b->amps);
    f(b->d_steps);
    f(b->d_ops);
    for (auto *w : b->d_work) f(w);
    b->d_work.clear();
    b->phase_blocks.clear();
    for (auto *w : b->d_work_reg) f(w);
    b->d_work_reg.clear();
    b->phase_blocks_reg.clear();
    f(b->d_phases);
    b->d_phases = nullptr;
    f(b->d_bm_circ);
    f(b->d_bm_start);
    f(b->d_init_blocks);
    b->d_init_blocks = nullptr;
    b->init_blocks = 0;
    f(b->d_offs);
    f(b->d_nq);
    f(b->d_term_off);
    f(b->d_terms);
    f(b->d_first_block);
    f(b->d_epart);
    f(b->d_energy);
    f(b->d_gpart);
    f(b->d_gop);
    f(b->d_gfirst);
    f(b->d_params);
    f(b->d_trig);
    if (b->h_energy) (void)hipHostFree(b->h_energy);
    if (b->h_gop) (void)hipHostFree(b->h_gop);
    if (b->h_params) (void)hipHostFree(b->h_params);
    b->amps = nullptr;
    b->d_steps = nullptr;
    b->d_ops = nullptr;
    b->d_bm_circ = nullptr;
    b->d_bm_start = nullptr;
    b->d_offs = nullptr;
    b->d_nq = nullptr;
    b->d_term_off = nullptr;
    b->d_terms = nullptr;
    b->d_first_block = nullptr;
    b->d_epart = b->d_energy = b->h_energy = nullptr;
    b->d_gpart = b->d_gop = b->h_gop = nullptr;
    b->d_gfirst = nullptr;
    b->d_params = b->h_params = nullptr;
    b->d_trig = nullptr;
    b->compiled = false;
}

// ---- run-time specialised register-path steps --------------------------------------
//
// A register-path step is a program: its tile size, phases and operators.
// Circuits of the same structure (the same qubit count and gate layout, any
// parameters) share their programs.  For every launch index s, one forward
// and one backward kernel switch over the programs of the s-th steps; each
// program is the generic kernel's code with its phases and operators as
// compile-time records (batch_dev.hpp), so operator dispatch, operator-field
// loads and the register copies where the dispatch arms meet disappear.
// Angles stay run-time values (the trig table), as do the step's placement
// (its DStep) and the gradient partials' addresses.

constexpr int kMaxPrograms = 512;
constexpr size_t kMaxProgramOps = 1u << 16;   // operator records over all programs

static std::string jit_hexd(double v)
{
    char buf[64];
    std::snprintf(buf, sizeof buf, "%a", v);
    return buf;
}

// The fields of an operator that its register-path code reads.
static std::string dop_init(const DOp &o)
{
    std::ostringstream s;
    const bool cz = o.kind == BOP_CZ, rot = o.kind == BOP_ROT, gate = o.kind == BOP_GATE;
    s << "{" << o.kind << ", " << o.pos0 << ", " << o.pos1 << ", " << (cz ? o.q0 : 0) << ", " << (cz ? o.q1 : 0)
      << ", " << (rot ? o.pauli : 0) << ", 0, " << (o.grad >= 0 ? 0 : -1) << ", 0ull, " << o.rbit << ", " << o.rbit1
      << ", " << (cz ? o.czrun : 0) << ", " << (o.grad >= 0 ? o.slot : 0) << ", 0.0, {";
    for (int i = 0; i < 8; i++) s << (i ? ", " : "") << (gate ? jit_hexd(o.m[i]) : std::string("0.0"));
    s << "}}";
    return s.str();
}

static bool phase_has_grads(const qs_batch *b, const BPhase &P)
{
    for (int k = P.op_begin; k < P.op_end; k++)
        if (b->h_ops[k].grad >= 0) return true;
    return false;
}

// Program key of register-path step si: everything its generated code
// depends on.
static std::string program_key(const qs_batch *b, int si)
{
    const DStep &st = b->h_steps[si];
    std::ostringstream k;
    k << st.qn << ";";
    for (int p = st.ph_begin; p < st.ph_end; p++) {
        const BPhase &P = b->h_phases[p];
        k << "P" << P.lo[0] << "," << P.lo[1] << "," << P.lo[2] << "," << P.rc[0] << "," << P.rc[1] << ","
          << P.rc[2] << "," << P.op_begin - st.op_begin << "," << P.op_end - st.op_begin << ";";
        for (int j = P.op_begin; j < P.op_end; j++) k << dop_init(b->h_ops[j]) << ";";
    }
    return k.str();
}

static void program_source(std::ostringstream &o, const qs_batch *b, int id, int si, bool bwd)
{
    const DStep &st = b->h_steps[si];
    const int np = st.ph_end - st.ph_begin;
    const unsigned nthr = 1u << (st.qn - 3);
    std::ostringstream ph;
    for (int k = 0; k < np; k++) {
        const BPhase &P = b->h_phases[st.ph_begin + k];
        ph << "    constexpr qs::BPhase P" << k << " = {{" << P.lo[0] << "u, " << P.lo[1] << "u, " << P.lo[2]
           << "u}, {" << P.rc[0] << ", " << P.rc[1] << ", " << P.rc[2] << "}, " << P.op_begin - st.op_begin << ", "
           << P.op_end - st.op_begin << "};\n";
    }
    auto op_line = [&](int j, const char *call) {
        o << "        { constexpr qs::DOp O = " << dop_init(b->h_ops[j]) << "; " << call << "(x, "
          << (bwd ? "y, " : "") << "O, st.op_begin + " << j - st.op_begin << ", trig, tau, base, czm"
          << (bwd ? ", red, lane, wave" : "") << "); }\n";
    };
    if (!bwd) {
        o << "template <typename R>\n__device__ __forceinline__ void bfwd_" << id
          << "(qs::C2<R> *__restrict__ amps, const qs::DStep &st, uint64_t base, const double *__restrict__ trig, "
             "unsigned char *lds)\n{\n"
          << ph.str();
        o << "    qs::C2<R> *v = reinterpret_cast<qs::C2<R> *>(lds);\n    qs::C2<R> *a = amps + st.amp_off;\n";
        o << "    const bool active = threadIdx.x < " << nthr << "u;\n";
        o << "    uint32_t tau = qs::bphase_tau(threadIdx.x, P0);\n    qs::C2<R> x[8];\n";
        o << "    if (active) {\n        const uint64_t xo = base | qs::tile_offset_bits(tau, st);\n"
             "        const qs::RegOffsets ro(P0, st);\n#pragma unroll\n"
             "        for (int u = 0; u < 8; u++) x[u] = qs::load_amp<R>(a, xo | ro(u), st.first);\n    }\n";
        for (int k = 0; k < np; k++) {
            const BPhase &P = b->h_phases[st.ph_begin + k];
            if (k) o << "    tau = qs::bphase_exchange<R>(x, v, tau, P" << k - 1 << ", P" << k << ", active);\n";
            o << "    if (active) {\n        uint32_t czm = 0;\n";
            for (int j = P.op_begin; j < P.op_end; j++) op_line(j, "qs::fwd_op<R>");
            o << "        (void)czm;\n    }\n";
        }
        o << "    if (active) {\n        const uint64_t xo = base | qs::tile_offset_bits(tau, st);\n"
             "        const qs::RegOffsets ro(P"
          << np - 1 << ", st);\n#pragma unroll\n        for (int u = 0; u < 8; u++) a[xo | ro(u)] = x[u];\n    }\n}\n\n";
        return;
    }
    o << "template <typename R>\n__device__ __forceinline__ void bbwd_" << id
      << "(qs::C2<R> *__restrict__ amps, uint64_t lambda_base, const qs::DStep &st, uint32_t tile, uint64_t base, "
         "const qs::DOp *__restrict__ ops, const double *__restrict__ trig, double *__restrict__ gpart, "
         "unsigned char *lds, double (*red)[qs::kRedRows])\n{\n"
      << ph.str();
    o << "    qs::C2<R> *vphi = reinterpret_cast<qs::C2<R> *>(lds);\n    qs::C2<R> *vlam = vphi + " << (1u << st.qn)
      << ";\n    qs::C2<R> *a = amps + st.amp_off;\n    qs::C2<R> *l = amps + lambda_base + st.amp_off;\n";
    o << "    const uint32_t t = threadIdx.x;\n    const bool active = t < " << nthr
      << "u;\n    const int lane = t & 63, wave = t >> 6;\n";
    o << "    uint32_t tau = qs::bphase_tau(t, P" << np - 1 << ");\n    qs::C2<R> x[8], y[8];\n";
    o << "    if (active) {\n        const uint64_t xo = base | qs::tile_offset_bits(tau, st);\n"
         "        const qs::RegOffsets ro(P"
      << np - 1
      << ", st);\n#pragma unroll\n        for (int u = 0; u < 8; u++) {\n            const uint64_t o = xo | ro(u);\n"
         "            x[u] = a[o];\n            y[u] = l[o];\n        }\n    }\n";
    auto flush = [&](int k) {
        const BPhase &D = b->h_phases[st.ph_begin + k];
        if (phase_has_grads(b, D))
            o << "    qs::flush_phase(ops, st.op_begin + " << D.op_begin - st.op_begin << ", st.op_begin + "
              << D.op_end - st.op_begin << ", red, " << (nthr >> 6) << ", tile, gpart);\n";
    };
    for (int k = np - 1; k >= 0; k--) {
        const BPhase &P = b->h_phases[st.ph_begin + k];
        if (k < np - 1) {
            o << "    __syncthreads();\n";
            flush(k + 1);
            o << "    tau = qs::bphase_exchange2<R>(x, y, vphi, vlam, tau, P" << k + 1 << ", P" << k << ", active);\n";
        }
        o << "    if (active) {\n        uint32_t czm = 0;\n";
        for (int j = P.op_end - 1; j >= P.op_begin; j--) op_line(j, "qs::bwd_op<R>");
        o << "        (void)czm;\n    }\n";
    }
    o << "    __syncthreads();\n";
    flush(0);
    o << "    if (active) {\n        const uint64_t xo = base | qs::tile_offset_bits(tau, st);\n"
         "        const qs::RegOffsets ro(P0, st);\n#pragma unroll\n        for (int u = 0; u < 8; u++) {\n"
         "            const uint64_t o = xo | ro(u);\n            a[o] = x[u];\n            l[o] = y[u];\n"
         "        }\n    }\n}\n\n";
}

// Source of the forward (bwd = false) or backward kernel of launch index s:
// the programs `progs` (id, representative step) and a switch over them.
static std::string launch_source(const qs_batch *b, int s, const std::vector<std::pair<int, int>> &progs, bool bwd)
{
    const bool f32 = b->precision == QS_C64;
    const char *c2 = f32 ? "float2" : "double2";
    std::ostringstream o;
    o << "#include \"batch_dev.hpp\"\n\n";
    for (const auto &pr : progs) program_source(o, b, pr.first, pr.second, bwd);
    if (!bwd) {
        o << "extern \"C\" __global__ __launch_bounds__(512) void qs_bfwd_" << s << "(" << c2
          << " *__restrict__ amps, const qs::DStep *__restrict__ steps, const uint2 *__restrict__ work, "
             "const double *__restrict__ trig)\n{\n";
    } else {
        o << "extern \"C\" __global__ __launch_bounds__(512) void qs_bbwd_" << s << "(" << c2
          << " *__restrict__ amps, unsigned long long lambda_base, const qs::DStep *__restrict__ steps, "
             "const qs::DOp *__restrict__ ops, const uint2 *__restrict__ work, const double *__restrict__ trig, "
             "double *__restrict__ gpart)\n{\n    __shared__ double red[qs::kPhaseRotMax][qs::kRedRows];\n";
    }
    o << "    using R = " << (f32 ? "float" : "double") << ";\n    extern __shared__ unsigned char lds_raw[];\n";
    o << "    const uint2 w = work[blockIdx.x];\n    const qs::DStep &st = steps[w.x];\n"
         "    const uint64_t base = qs::insert_zeros(w.y, st.plan);\n    switch (st.prog) {\n";
    for (const auto &pr : progs) {
        if (!bwd)
            o << "    case " << pr.first << ": bfwd_" << pr.first << "<R>(amps, st, base, trig, lds_raw); break;\n";
        else
            o << "    case " << pr.first << ": bbwd_" << pr.first
              << "<R>(amps, lambda_base, st, w.y, base, ops, trig, gpart, lds_raw, red); break;\n";
    }
    o << "    default: break;\n    }\n}\n";
    return o.str();
}

static int specialize_batch(qs_batch *b, int *num_programs)
{
    // programs of the register-path steps
    std::map<std::string, int> ids;
    std::vector<int> prog_of(b->h_steps.size(), -1);
    std::vector<int> rep;   // representative step of every program
    size_t total_ops = 0;
    int launches = 0;
    for (size_t si = 0; si < b->h_steps.size(); si++) {
        const DStep &st = b->h_steps[si];
        if (st.qn < kRegMinQubits) continue;
        const std::string key = program_key(b, (int)si);
        auto it = ids.find(key);
        if (it == ids.end()) {
            it = ids.emplace(key, (int)rep.size()).first;
            rep.push_back((int)si);
            total_ops += (size_t)(st.op_end - st.op_begin);
        }
        prog_of[si] = it->second;
        launches = std::max(launches, b->step_launch[si] + 1);
    }
    if (num_programs) *num_programs = (int)rep.size();
    if (rep.empty()) return QS_OK;
    if ((int)rep.size() > kMaxPrograms || total_ops > kMaxProgramOps)
        return fail(QS_E_PRECOND, "too many distinct step programs to specialise (" + std::to_string(rep.size()) +
                                      " programs, " + std::to_string(total_ops) + " operators)");
    // per launch index, the programs its steps use
    std::vector<std::vector<std::pair<int, int>>> per_launch(launches);
    {
        std::vector<std::vector<char>> seen(launches, std::vector<char>(rep.size(), 0));
        for (size_t si = 0; si < b->h_steps.size(); si++) {
            const int pg = prog_of[si];
            if (pg < 0) continue;
            const int s = b->step_launch[si];
            if (!seen[s][pg]) {
                seen[s][pg] = 1;
                per_launch[s].push_back({pg, rep[pg]});
            }
        }
    }
    std::vector<std::string> srcs;
    std::vector<std::pair<int, bool>> src_of;   // (launch, backward)
    for (int s = 0; s < launches; s++) {
        if (per_launch[s].empty()) continue;
        for (bool bwd : {false, true}) {
            srcs.push_back(launch_source(b, s, per_launch[s], bwd));
            src_of.push_back({s, bwd});
        }
    }
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QS_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::vector<std::vector<char>> codes;
    int rc = compile_device_sources(srcs, arch, codes);
    if (rc != QS_OK) return rc;

    // the graphs hold the kernels they were captured with: both go, and the
    // graphs are captured again with whichever kernels remain
    QS_HIP(hipStreamSynchronize(b->stream));
    if (b->g_fwd) (void)hipGraphExecDestroy(b->g_fwd);
    if (b->g_full) (void)hipGraphExecDestroy(b->g_full);
    if (b->gr_fwd) (void)hipGraphDestroy(b->gr_fwd);
    if (b->gr_full) (void)hipGraphDestroy(b->gr_full);
    b->g_fwd = b->g_full = nullptr;
    b->gr_fwd = b->gr_full = nullptr;
    release_jit(b);
    auto recapture = [&]() {
        int r = QS_OK;
        if (b->use_graph && (r = capture(b, false, &b->gr_fwd, &b->g_fwd)) == QS_OK)
            r = capture(b, true, &b->gr_full, &b->g_full);
        if (r != QS_OK) b->compiled = false;
        return r;
    };
    auto give_up = [&](const std::string &msg) {
        const std::string m = msg;   // the generic kernels again
        release_jit(b);
        recapture();
        return fail(QS_E_HIP, m);
    };
    std::vector<void *> fwd(launches, nullptr), bwd_k(launches, nullptr);
    for (size_t k = 0; k < codes.size(); k++) {
        hipModule_t mod;
        if (hipModuleLoadData(&mod, codes[k].data()) != hipSuccess) {
            (void)hipGetLastError();
            return give_up("loading the specialised batch steps failed");
        }
        b->jit_modules.push_back(mod);
        const int s = src_of[k].first;
        const bool bwd = src_of[k].second;
        const std::string name = (bwd ? "qs_bbwd_" : "qs_bfwd_") + std::to_string(s);
        hipFunction_t f = nullptr;
        if (hipModuleGetFunction(&f, mod, name.c_str()) != hipSuccess) {
            (void)hipGetLastError();
            return give_up("specialised kernel " + name + " missing from its module");
        }
        (bwd ? bwd_k : fwd)[s] = (void *)f;
    }
    // the steps' program numbers
    for (size_t si = 0; si < b->h_steps.size(); si++) b->h_steps[si].prog = prog_of[si];
    if (hipMemcpy(b->d_steps, b->h_steps.data(), b->h_steps.size() * sizeof(DStep), hipMemcpyHostToDevice) !=
        hipSuccess) {
        (void)hipGetLastError();
        return give_up("uploading the step table failed");
    }
    b->jit_fwd = fwd;
    b->jit_bwd = bwd_k;
    b->num_programs = (int)rep.size();
    return recapture();
}

}  // namespace qs

extern "C" {

int qs_batch_create(int precision, qs_batch **out)
{
    if (!out) return fail(QS_E_ARG, "null output pointer");
    if (precision != QS_C64 && precision != QS_C128) return fail(QS_E_ARG, "bad precision");
    qs_batch *b = new (std::nothrow) qs_batch{};
    if (!b) return fail(QS_E_ALLOC, "host allocation failed");
    b->precision = precision;
    b->tile_qubits = precision == QS_C64 ? 12 : 11;
    b->low_qubits = precision == QS_C64 ? 3 : 2;
    *out = b;
    return QS_OK;
}

int qs_batch_destroy(qs_batch *b)
{
    if (!b) return QS_OK;
    if (b->compiled) (void)hipStreamSynchronize(b->stream);
    release(b);
    delete b;
    return QS_OK;
}

int qs_batch_add_circuit(qs_batch *b, int num_qubits, int num_params, int *index)
{
    if (!b) return fail(QS_E_ARG, "null batch");
    if (num_qubits < 1 || num_qubits > 30) return fail(QS_E_ARG, "batch circuits have 1 to 30 qubits");
    if (num_params < 0) return fail(QS_E_ARG, "negative parameter count");
    BCirc c{};
    c.n = num_qubits;
    c.num_params = num_params;
    b->circs.push_back(std::move(c));
    b->compiled = false;
    if (index) *index = (int)b->circs.size() - 1;
    return QS_OK;
}

static BCirc *circ_at(qs_batch *b, int i)
{
    if (!b || i < 0 || i >= (int)b->circs.size()) return nullptr;
    return &b->circs[i];
}

int qs_batch_add_rotation(qs_batch *b, int circuit, int qubit, int pauli, int param, double scale)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (qubit < 0 || qubit >= c->n) return fail(QS_E_ARG, "qubit out of range");
    if (pauli < 1 || pauli > 3) return fail(QS_E_ARG, "rotation Pauli is 1 (X), 2 (Y) or 3 (Z)");
    if (param < 0 || param >= c->num_params) return fail(QS_E_ARG, "parameter index out of range");
    BOp op{};
    op.kind = BOP_ROT;
    op.q0 = qubit;
    op.q1 = qubit;
    op.pauli = pauli;
    op.param = param;
    op.scale = scale;
    c->ops.push_back(op);
    b->compiled = false;
    return QS_OK;
}

int qs_batch_add_gate1(qs_batch *b, int circuit, int qubit, const double *m)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (!m) return fail(QS_E_ARG, "null matrix");
    if (qubit < 0 || qubit >= c->n) return fail(QS_E_ARG, "qubit out of range");
    BOp op{};
    op.kind = BOP_GATE;
    op.q0 = qubit;
    op.q1 = qubit;
    for (int k = 0; k < 4; k++) op.m[k] = cd(m[2 * k], m[2 * k + 1]);
    c->ops.push_back(op);
    b->compiled = false;
    return QS_OK;
}

// A Pauli gadget exp(i theta P) on several qubits (Sec. "Pauli gadget") as
// the rotation exp(i theta X_w) on one of its qubits w between Clifford
// gates: exp(i theta P) = B^dag exp(i theta Z_S) B with B the per-qubit basis
// change (H for X, H S^dag for Y) that turns P into Z_S on its support S, and
// exp(i theta Z_S) = L exp(i theta Z_w) L with L the CNOTs from every other
// qubit of S onto w (L Z_w L = Z_S); CNOT(c, w) = H_w CZ(c, w) H_w and
// H_w exp(i theta Z_w) H_w = exp(i theta X_w).  In circuit order: H_w B_w on
// w and B_q on the others, the CZs, the rotation, the CZs, B^dag and H_w.
// The Clifford gates do not depend on theta, so the adjoint sweep's
// derivative of the rotation is the gadget's.
static int add_gadget(qs_batch *b, BCirc *c, const int *targs, const int *paulis, int n, int param, double scale)
{
    std::vector<int> q, pc;
    for (int k = 0; k < n; k++) {
        if (targs[k] < 0 || targs[k] >= c->n) return fail(QS_E_ARG, "qubit out of range");
        if (paulis[k] < 0 || paulis[k] > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
        for (int j = 0; j < k; j++)
            if (targs[j] == targs[k]) return fail(QS_E_ARG, "duplicate qubit");
        if (paulis[k]) {
            q.push_back(targs[k]);
            pc.push_back(paulis[k]);
        }
    }
    if (q.empty()) return fail(QS_E_ARG, "an identity string is a global phase, not a gadget");
    if (param >= c->num_params) return fail(QS_E_ARG, "parameter index out of range");
    const double r = 1.0 / std::sqrt(2.0);
    const cd I(0, 1);
    const cd H[4] = {r, r, r, -r};
    const cd BY[4] = {r, -I * r, r, I * r};          // H S^dag
    const cd BYd[4] = {r, r, I * r, -I * r};         // (H S^dag)^dag
    const cd SD[4] = {1, 0, 0, -I};                  // S^dag
    const cd S[4] = {1, 0, 0, I};
    auto gate = [&](int qubit, const cd *m) {
        BOp op{};
        op.kind = BOP_GATE;
        op.q0 = op.q1 = qubit;
        for (int k = 0; k < 4; k++) op.m[k] = m[k];
        op.logical = 0;
        c->ops.push_back(op);
    };
    auto cz = [&](int a, int w) {
        BOp op{};
        op.kind = BOP_CZ;
        op.q0 = a;
        op.q1 = w;
        op.logical = 0;
        c->ops.push_back(op);
    };
    const size_t wi = q.size() - 1;   // the rotation's qubit
    const int w = q[wi];
    // basis changes (pivot: H_w B_w = I for X, S^dag for Y, H for Z)
    for (size_t k = 0; k < q.size(); k++) {
        if (k == wi) {
            if (pc[k] == 2) gate(w, SD);
            else if (pc[k] == 3) gate(w, H);
        } else if (pc[k] == 1) {
            gate(q[k], H);
        } else if (pc[k] == 2) {
            gate(q[k], BY);
        }
    }
    for (size_t k = 0; k < wi; k++) cz(q[k], w);
    BOp rot{};
    if (param >= 0) {
        rot.kind = BOP_ROT;
        rot.pauli = 1;
        rot.param = param;
        rot.scale = scale;
    } else {
        // fixed angle: exp(i scale X) as a gate
        rot.kind = BOP_GATE;
        const double co = std::cos(scale), si = std::sin(scale);
        rot.m[0] = co;
        rot.m[1] = I * si;
        rot.m[2] = I * si;
        rot.m[3] = co;
    }
    rot.q0 = rot.q1 = w;
    c->ops.push_back(rot);
    for (size_t k = 0; k < wi; k++) cz(q[k], w);
    for (size_t k = 0; k < q.size(); k++) {
        if (k == wi) {
            if (pc[k] == 2) gate(w, S);
            else if (pc[k] == 3) gate(w, H);
        } else if (pc[k] == 1) {
            gate(q[k], H);
        } else if (pc[k] == 2) {
            gate(q[k], BYd);
        }
    }
    b->compiled = false;
    return QS_OK;
}

int qs_batch_add_gadget(qs_batch *b, int circuit, const int *targs, const int *paulis, int num_targs, int param,
                        double scale)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (num_targs < 1 || !targs || !paulis) return fail(QS_E_ARG, "empty Pauli string");
    return add_gadget(b, c, targs, paulis, num_targs, param, scale);
}

int qs_batch_add_cz(qs_batch *b, int circuit, int q1, int q2)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (q1 < 0 || q1 >= c->n || q2 < 0 || q2 >= c->n || q1 == q2) return fail(QS_E_ARG, "bad CZ qubits");
    BOp op{};
    op.kind = BOP_CZ;
    op.q0 = q1;
    op.q1 = q2;
    c->ops.push_back(op);
    b->compiled = false;
    return QS_OK;
}

int qs_batch_set_observable(qs_batch *b, int circuit, const int *paulis, const double *coeffs, int num_terms)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (num_terms < 0 || (num_terms > 0 && (!paulis || !coeffs))) return fail(QS_E_ARG, "bad observable");
    for (int i = 0; i < num_terms * c->n; i++)
        if (paulis[i] < 0 || paulis[i] > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
    c->codes.assign(paulis, paulis + (size_t)num_terms * c->n);
    c->coeffs.assign(coeffs, coeffs + num_terms);
    b->compiled = false;
    return QS_OK;
}

int qs_batch_compile(qs_batch *b, void *hip_stream, int use_graph)
{
    if (!b) return fail(QS_E_ARG, "null batch");
    if (b->circs.empty()) return fail(QS_E_ARG, "empty batch");
    if (b->compiled) (void)hipStreamSynchronize(b->stream);
    release(b);
    b->use_graph = use_graph ? 1 : 0;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        // the legacy null stream cannot be captured: use a stream of our own
        // (default priority)
        QS_HIP(hipStreamCreate(&b->stream));
        b->own_stream = true;
    }
    const size_t ab = b->precision == QS_C64 ? 8 : 16;
    {
        // the adjoint sweep holds two tiles in LDS
        int dev = 0, max_lds = 0;
        QS_HIP(hipGetDevice(&dev));
        QS_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        b->tile_qubits = b->precision == QS_C64 ? 12 : 11;
        // the adjoint sweep's two tiles and its partial sums
        const size_t red = sizeof(double) * kPhaseRotMax * kRedRows;
        while (b->tile_qubits > b->low_qubits + 1 && (2 * ((size_t)1 << b->tile_qubits) * ab + red) > (size_t)max_lds)
            b->tile_qubits--;
    }
    const int TQ = b->tile_qubits, C = b->low_qubits;

    // layout: each circuit's amplitudes start on a 256-amplitude boundary
    uint64_t off = 0;
    int poff = 0;
    size_t max_steps = 0;
    for (auto &c : b->circs) {
        plan_circuit(c, TQ, C);
        c.amp_off = off;
        off += ((1ULL << c.n) + 255) & ~255ULL;
        c.param_off = poff;
        poff += c.num_params;
        max_steps = std::max(max_steps, c.steps.size());
    }
    b->total_amps = off;
    b->total_params = poff;
    // per-amplitude launches cover the whole batch in one dispatch, whose
    // size in work-items is a 32-bit number
    if (off > 0xFFFFFFFFull - 255) return fail(QS_E_ARG, "batch holds more than 2^32 amplitudes");

    // steps, operators, rotation slots and gradient partials
    std::vector<DStep> steps;
    std::vector<DOp> ops;
    std::vector<BPhase> phases;
    b->step_launch.clear();
    std::vector<uint64_t> gfirst{0};
    b->rot_param.clear();
    b->rot_scale.clear();
    std::vector<std::vector<int>> step_index(b->circs.size());
    for (size_t ci = 0; ci < b->circs.size(); ci++) {
        BCirc &c = b->circs[ci];
        for (auto &s : c.steps) {
            DStep d{};
            d.prog = -1;
            d.first = step_index[ci].empty() ? 1 : 0;
            d.amp_off = c.amp_off;
            std::vector<int> qs_;
            for (int q = 0; q < c.n; q++)
                if ((s.qmask >> q) & 1) qs_.push_back(q);
            d.plan = make_insert_plan(qs_);
            d.qn = (int)qs_.size();
            for (int k = 0; k < d.qn; k++) d.qpos[k] = qs_[k];
            d.op_begin = (int)ops.size();
            const uint64_t tiles = 1ULL << (c.n - d.qn);
            for (int k : s.ops) {
                const BOp &o = c.ops[k];
                DOp x{};
                x.kind = o.kind;
                x.q0 = o.q0;
                x.q1 = o.q1;
                auto pos = [&](int q) {
                    auto it = std::find(qs_.begin(), qs_.end(), q);
                    return it == qs_.end() ? -1 : (int)(it - qs_.begin());
                };
                x.pos0 = pos(o.q0);
                x.pos1 = pos(o.q1);
                x.pauli = o.pauli;
                x.param = c.param_off + o.param;
                x.scale = o.scale;
                for (int m = 0; m < 4; m++) {
                    x.m[2 * m] = o.m[m].real();
                    x.m[2 * m + 1] = o.m[m].imag();
                }
                x.grad = -1;
                x.rbit = x.rbit1 = -1;
                if (o.kind == BOP_ROT) {
                    x.grad = (int)b->rot_param.size();
                    x.gpart = gfirst.back();
                    gfirst.push_back(gfirst.back() + tiles);
                    b->rot_param.push_back(c.param_off + o.param);
                    b->rot_scale.push_back(o.scale);
                }
                ops.push_back(x);
            }
            d.op_end = (int)ops.size();
            d.ph_begin = d.ph_end = (int)phases.size();
            if (d.qn >= kRegMinQubits) {
                // register phases: at most 3 operator coordinates and
                // kPhaseRotMax rotations each; a phase takes, in order, every
                // remaining operator that fits it and shares no qubit with a
                // remaining operator it jumps over (the step's operators are
                // regrouped by phase)
                std::vector<DOp> seg(ops.begin() + d.op_begin, ops.begin() + d.op_end), out;
                std::vector<char> used(seg.size(), 0);
                auto support = [](const DOp &x) {
                    return (1ULL << x.q0) | (x.kind == BOP_CZ ? (1ULL << x.q1) : 0ULL);
                };
                while (out.size() < seg.size()) {
                    BPhase ph{};
                    std::vector<int> R;
                    int nrot = 0;
                    uint64_t blocked = 0;
                    const size_t first = out.size();
                    for (size_t i = 0; i < seg.size(); i++) {
                        if (used[i]) continue;
                        DOp x = seg[i];
                        const uint64_t sp = support(x);
                        bool fits = !(sp & blocked);
                        if (fits && x.kind != BOP_CZ) {
                            const bool in = std::find(R.begin(), R.end(), x.pos0) != R.end();
                            if ((!in && R.size() == 3) || (x.kind == BOP_ROT && nrot == kPhaseRotMax)) fits = false;
                            if (fits) {
                                if (!in) R.push_back(x.pos0);
                                if (x.kind == BOP_ROT) x.slot = nrot++;
                            }
                        }
                        if (fits) {
                            used[i] = 1;
                            out.push_back(x);
                        } else {
                            blocked |= sp;
                        }
                    }
                    ph.op_begin = d.op_begin + (int)first;
                    ph.op_end = d.op_begin + (int)out.size();
                    for (int cc = d.qn - 1; R.size() < 3; cc--)
                        if (std::find(R.begin(), R.end(), cc) == R.end()) R.push_back(cc);
                    std::vector<int> sorted_r = R;
                    std::sort(sorted_r.begin(), sorted_r.end());
                    for (int j = 0; j < 3; j++) {
                        ph.rc[j] = R[j];
                        ph.lo[j] = (1u << sorted_r[j]) - 1u;
                    }
                    auto rbit_of = [&](int pos) {
                        auto it = std::find(R.begin(), R.end(), pos);
                        return it == R.end() ? -1 : (int)(it - R.begin());
                    };
                    for (size_t kk = first; kk < out.size(); kk++) {
                        out[kk].rbit = rbit_of(out[kk].pos0);
                        out[kk].rbit1 = out[kk].kind == BOP_CZ ? rbit_of(out[kk].pos1) : -1;
                    }
                    // a CZ joins the phase's previous run of CZs when it
                    // commutes with every operator between them (no shared
                    // qubit, or a Z rotation: diagonal), so that the kernels
                    // apply each run as one sign mask
                    {
                        std::vector<DOp> ord;
                        for (size_t kk = first; kk < out.size(); kk++) {
                            const DOp &x = out[kk];
                            size_t at = ord.size();
                            if (x.kind == BOP_CZ) {
                                size_t j = ord.size();
                                while (j > 0 && ord[j - 1].kind != BOP_CZ) {
                                    const DOp &o = ord[j - 1];
                                    if ((support(o) & support(x)) && !(o.kind == BOP_ROT && o.pauli == 3)) break;
                                    j--;
                                }
                                if (j > 0 && ord[j - 1].kind == BOP_CZ) at = j;
                            }
                            ord.insert(ord.begin() + (long)at, x);
                        }
                        for (size_t kk = 0; kk < ord.size(); kk++) {
                            if (ord[kk].kind != BOP_CZ) continue;
                            ord[kk].czrun = (kk == 0 || ord[kk - 1].kind != BOP_CZ ? 1 : 0) |
                                            (kk + 1 == ord.size() || ord[kk + 1].kind != BOP_CZ ? 2 : 0);
                        }
                        std::copy(ord.begin(), ord.end(), out.begin() + (long)first);
                    }
                    phases.push_back(ph);
                }
                std::copy(out.begin(), out.end(), ops.begin() + d.op_begin);
                d.ph_end = (int)phases.size();
            }
            step_index[ci].push_back((int)steps.size());
            b->step_launch.push_back((int)step_index[ci].size() - 1);
            steps.push_back(d);
        }
    }
    b->num_rot = (int)b->rot_param.size();

    // per-phase work lists: (step, tile) per block, register path or LDS path
    std::vector<std::vector<uint2>> work(max_steps), work_reg(max_steps);
    for (size_t ci = 0; ci < b->circs.size(); ci++) {
        const BCirc &c = b->circs[ci];
        for (size_t s = 0; s < c.steps.size(); s++) {
            const int si = step_index[ci][s];
            const uint64_t tiles = 1ULL << (c.n - steps[si].qn);
            auto &wl = steps[si].qn >= kRegMinQubits ? work_reg[s] : work[s];
            for (uint64_t t = 0; t < tiles; t++) wl.push_back(make_uint2((unsigned)si, (unsigned)t));
        }
    }

    // 256-amplitude block map, observables
    std::vector<int> bm_circ, first_block, nq, term_off{0};
    std::vector<uint64_t> bm_start, offs;
    std::vector<DTerm> terms;
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    for (size_t ci = 0; ci < b->circs.size(); ci++) {
        const BCirc &c = b->circs[ci];
        first_block.push_back((int)bm_circ.size());
        for (uint64_t s = 0; s < (1ULL << c.n); s += 256) {
            bm_circ.push_back((int)ci);
            bm_start.push_back(s);
        }
        offs.push_back(c.amp_off);
        nq.push_back(c.n);
        const int T = (int)c.coeffs.size();
        for (int t = 0; t < T; t++) {
            DTerm d{};
            int ny = 0;
            for (int q = 0; q < c.n; q++) {
                const int code = c.codes[(size_t)t * c.n + q];
                if (code == 1 || code == 2) d.x |= 1ULL << q;
                if (code == 2 || code == 3) d.yz |= 1ULL << q;
                if (code == 2) ny++;
            }
            const cd cf = c.coeffs[t] * eta[ny & 3];
            d.cre = cf.real();
            d.cim = cf.imag();
            terms.push_back(d);
        }
        // padded with zero terms to whole groups of the gather kernel
        while ((terms.size() - (size_t)term_off.back()) % kTermGroup) terms.push_back(DTerm{});
        term_off.push_back((int)terms.size());
    }
    first_block.push_back((int)bm_circ.size());
    b->amp_blocks = (unsigned)bm_circ.size();
    std::vector<int> init_blocks;
    for (size_t k = 0; k < bm_circ.size(); k++)
        if (b->circs[(size_t)bm_circ[k]].steps.empty()) init_blocks.push_back((int)k);
    b->init_blocks = (unsigned)init_blocks.size();

    int rc = QS_OK;
    auto up = [&](auto **dst, const auto &vec) {
        if (rc == QS_OK) rc = upload(dst, vec.data(), vec.size() * sizeof(vec[0]));
    };
    if (hipMalloc(&b->amps, 2 * b->total_amps * ab) != hipSuccess) {
        (void)hipGetLastError();
        b->amps = nullptr;
        return fail(QS_E_ALLOC, "device allocation of the batch states failed");
    }
    up(&b->d_steps, steps);
    up(&b->d_ops, ops);
    up(&b->d_bm_circ, bm_circ);
    up(&b->d_bm_start, bm_start);
    up(&b->d_init_blocks, init_blocks);
    up(&b->d_offs, offs);
    up(&b->d_nq, nq);
    up(&b->d_term_off, term_off);
    up(&b->d_terms, terms);
    up(&b->d_first_block, first_block);
    up(&b->d_gfirst, gfirst);
    if (rc != QS_OK) return rc;
    for (auto &w : work) {
        uint2 *d = nullptr;
        rc = upload(&d, w.data(), w.size() * sizeof(uint2));
        if (rc != QS_OK) return rc;
        b->d_work.push_back(d);
        b->phase_blocks.push_back((unsigned)w.size());
    }
    for (auto &w : work_reg) {
        uint2 *d = nullptr;
        rc = upload(&d, w.data(), w.size() * sizeof(uint2));
        if (rc != QS_OK) return rc;
        b->d_work_reg.push_back(d);
        b->phase_blocks_reg.push_back((unsigned)w.size());
    }
    up(&b->d_phases, phases);
    b->h_steps = steps;
    b->h_ops = ops;
    b->h_phases = phases;
    if (rc != QS_OK) return rc;
    if ((rc = upload(&b->d_epart, nullptr, sizeof(double) * 2 * bm_circ.size())) != QS_OK) return rc;
    if ((rc = upload(&b->d_energy, nullptr, sizeof(double) * 2 * b->circs.size())) != QS_OK) return rc;
    if ((rc = upload(&b->d_gpart, nullptr, sizeof(double) * std::max<uint64_t>(1, gfirst.back()))) != QS_OK) return rc;
    if ((rc = upload(&b->d_gop, nullptr, sizeof(double) * std::max(1, b->num_rot))) != QS_OK) return rc;
    if ((rc = upload(&b->d_params, nullptr, sizeof(double) * std::max(1, b->total_params))) != QS_OK) return rc;
    b->num_ops = (int)ops.size();
    if ((rc = upload(&b->d_trig, nullptr, sizeof(double) * 2 * std::max(1, b->num_ops))) != QS_OK) return rc;
    if (hipHostMalloc(&b->h_energy, sizeof(double) * 2 * b->circs.size(), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_gop, sizeof(double) * std::max(1, b->num_rot), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_params, sizeof(double) * std::max(1, b->total_params), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QS_E_ALLOC, "pinned host allocation failed");
    }
    if (b->use_graph) {
        if ((rc = capture(b, false, &b->gr_fwd, &b->g_fwd)) != QS_OK) return rc;
        if ((rc = capture(b, true, &b->gr_full, &b->g_full)) != QS_OK) return rc;
    }
    b->compiled = true;
    return QS_OK;
}

int qs_batch_run(qs_batch *b, const double *params, double *energies, double *grads)
{
    if (!b) return fail(QS_E_ARG, "null batch");
    if (!b->compiled) return fail(QS_E_PRECOND, "batch is not compiled");
    if (b->total_params > 0 && !params) return fail(QS_E_ARG, "null parameters");
    const bool want_grads = grads != nullptr;
    QS_HIP(hipStreamSynchronize(b->stream));
    if (b->total_params > 0) {
        std::memcpy(b->h_params, params, sizeof(double) * b->total_params);
        QS_HIP(hipMemcpyAsync(b->d_params, b->h_params, sizeof(double) * b->total_params, hipMemcpyHostToDevice,
                              b->stream));
    }
    if (b->use_graph) {
        QS_HIP(hipGraphLaunch(want_grads ? b->g_full : b->g_fwd, b->stream));
    } else {
        int rc = launch_phase_kernels(b, want_grads);
        if (rc != QS_OK) return rc;
    }
    QS_HIP(hipMemcpyAsync(b->h_energy, b->d_energy, sizeof(double) * 2 * b->circs.size(), hipMemcpyDeviceToHost,
                          b->stream));
    if (want_grads && b->num_rot > 0)
        QS_HIP(hipMemcpyAsync(b->h_gop, b->d_gop, sizeof(double) * b->num_rot, hipMemcpyDeviceToHost, b->stream));
    QS_HIP(hipStreamSynchronize(b->stream));
    if (energies)
        for (size_t c = 0; c < b->circs.size(); c++) energies[c] = b->h_energy[2 * c];
    if (want_grads) {
        for (int p = 0; p < b->total_params; p++) grads[p] = 0.0;
        // dE/dtheta_p += 2 Re(i scale <lambda|P|phi>) = -2 scale Im<lambda|P|phi>
        for (int r = 0; r < b->num_rot; r++) grads[b->rot_param[r]] += -2.0 * b->rot_scale[r] * b->h_gop[r];
    }
    b->last_run_had_grads = want_grads;
    return QS_OK;
}

int qs_batch_get_state(qs_batch *b, int circuit, double *re_im)
{
    BCirc *c = circ_at(b, circuit);
    if (!c) return fail(QS_E_ARG, "no such circuit");
    if (!b->compiled) return fail(QS_E_PRECOND, "batch is not compiled");
    if (!re_im) return fail(QS_E_ARG, "null output");
    QS_HIP(hipStreamSynchronize(b->stream));
    const uint64_t n = 1ULL << c->n;
    if (b->precision == QS_C128) {
        QS_HIP(hipMemcpy(re_im, (double2 *)b->amps + c->amp_off, n * 16, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * n);
        QS_HIP(hipMemcpy(tmp.data(), (float2 *)b->amps + c->amp_off, n * 8, hipMemcpyDeviceToHost));
        for (uint64_t i = 0; i < 2 * n; i++) re_im[i] = tmp[i];
    }
    return QS_OK;
}

int qs_batch_stats(const qs_batch *b, int *num_circuits, int *num_steps, uint64_t *total_amps,
                   uint64_t *logical_updates)
{
    if (!b) return fail(QS_E_ARG, "null batch");
    if (num_circuits) *num_circuits = (int)b->circs.size();
    if (num_steps) *num_steps = (int)b->d_work.size();
    uint64_t amps = 0, upd = 0;
    for (const auto &c : b->circs) {
        amps += 1ULL << c.n;
        uint64_t n_ops = 0;
        for (const auto &op : c.ops) n_ops += (uint64_t)op.logical;
        upd += n_ops << c.n;
    }
    if (total_amps) *total_amps = amps;
    if (logical_updates) *logical_updates = upd;
    return QS_OK;
}

int qs_batch_specialize(qs_batch *b, int *num_programs)
{
    if (!b) return fail(QS_E_ARG, "null batch");
    if (!b->compiled) return fail(QS_E_PRECOND, "batch is not compiled");
    return specialize_batch(b, num_programs);
}

}  // extern "C"
