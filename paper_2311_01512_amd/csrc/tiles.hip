// LDS tile engine for recorded circuits.
//
// A step owns a subspace span(W) of the index space (GF(2) vectors, at most
// T dimensions) that always contains the unit vectors of the lowest C
// qubits, so each tile is read in runs of 2^C consecutive amplitudes (a full
// 128-byte line).  A dense gate fits a step when the unit vectors of its
// targets lie in span(W); a Pauli gadget fits when its X/Y flip mask does,
// whatever its weight, since the gadget only pairs i with i ^ x.  Each tile
// (coset base ^ span(W)) is gathered into LDS, every operator of the step is
// applied there in order, and the tile is written back: one HBM pass for
// the whole step.  Operators join a step only if they commute with every
// operator they jump over (no shared qubit), so the circuit's order holds.
#include "circuit.hpp"

#include <algorithm>
#include <map>

namespace qs {

// ---- GF(2) reduced echelon basis ----------------------------------------------------

struct Echelon {
    std::map<int, uint64_t> by_pivot;   // pivot bit -> vector (pivot = highest set bit)

    uint64_t reduce(uint64_t x) const
    {
        for (auto it = by_pivot.rbegin(); it != by_pivot.rend(); ++it)
            if ((x >> it->first) & 1ULL) x ^= it->second;
        return x;
    }
    // Adds x; keeps every pivot bit set in exactly one vector.
    bool add(uint64_t x)
    {
        x = reduce(x);
        if (!x) return false;
        const int p = 63 - __builtin_clzll(x);
        for (auto &kv : by_pivot)
            if ((kv.second >> p) & 1ULL) kv.second ^= x;
        by_pivot[p] = x;
        return true;
    }
    int dim() const { return (int)by_pivot.size(); }
    int dim_with(const std::vector<uint64_t> &xs) const
    {
        Echelon e = *this;
        for (uint64_t x : xs) e.add(x);
        return e.dim();
    }
};

static bool absorbable(const CircOp &op) { return op.gadget || op.targs.size() <= 3; }

static std::vector<uint64_t> needed_vectors(const CircOp &op)
{
    std::vector<uint64_t> v;
    if (op.gadget) {
        uint64_t x = 0;
        for (size_t k = 0; k < op.targs.size(); k++)
            if (op.paulis[k] == 1 || op.paulis[k] == 2) x |= 1ULL << op.targs[k];
        if (x) v.push_back(x);
    } else {
        for (int t : op.targs) v.push_back(1ULL << t);
    }
    return v;
}

static uint64_t support_mask(const CircOp &op)
{
    uint64_t s = 0;
    for (int q : op.support()) s |= 1ULL << q;
    return s;
}

int tile_dim_limit(int precision)
{
    int dev = 0, max_lds = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        max_lds = 65536;
    }
    const size_t ab = precision == QS_C64 ? 8 : 16;
    int d = kTileDimMax;
    while (d > 1 && ((size_t)1 << d) * ab > (size_t)max_lds) d--;
    return d;
}

// Operators of a finished step in the step's coordinates.
static void encode_step(Pass &p, const Echelon &E, const std::vector<const CircOp *> &members)
{
    p.tile = true;
    p.gadget = false;
    p.basis.clear();
    p.pivots.clear();
    for (auto &kv : E.by_pivot) {
        p.pivots.push_back(kv.first);
        p.basis.push_back(kv.second);
    }
    p.tile_d = (int)p.basis.size();
    auto coord_of_pivot = [&](int b) {
        return (int)(std::find(p.pivots.begin(), p.pivots.end(), b) - p.pivots.begin());
    };
    auto qubit_mask = [&](int b) {
        uint32_t m = 0;
        for (int k = 0; k < p.tile_d; k++)
            if ((p.basis[k] >> b) & 1ULL) m |= 1u << k;
        return m;
    };
    auto flip_of = [&](uint64_t x) {
        uint32_t f = 0;
        for (int k = 0; k < p.tile_d; k++)
            if ((x >> p.pivots[k]) & 1ULL) f |= 1u << k;
        return f;
    };
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    p.tops.clear();
    p.tmats.clear();
    for (const CircOp *op : members) {
        TOp t{};
        if (op->gadget) {
            t.kind = 1;
            uint64_t x = 0, yz = 0;
            int ny = 0;
            for (size_t k = 0; k < op->targs.size(); k++) {
                const int c = op->paulis[k];
                const uint64_t b = 1ULL << op->targs[k];
                if (c == 1 || c == 2) x |= b;
                if (c == 2 || c == 3) yz |= b;
                if (c == 2) ny++;
            }
            t.flip = flip_of(x);
            t.yz = yz;
            uint32_t ym = 0;
            for (int b = 0; b < 64; b++)
                if ((yz >> b) & 1ULL) ym ^= qubit_mask(b);
            t.yzm = ym;
            const cd c = cd(0, std::sin(op->theta)) * eta[ny & 3];
            t.cs = std::cos(op->theta);
            t.cre = c.real();
            t.cim = c.imag();
        } else {
            t.kind = 0;
            std::vector<int> sorted;
            std::vector<cd> Ms = permute_to_sorted(op->M, op->targs, sorted);
            t.nt = (int)sorted.size();
            for (int i = 0; i < t.nt; i++) t.pos[i] = coord_of_pivot(sorted[i]);
            t.nc = (int)op->ctrls.size();
            for (int i = 0; i < t.nc; i++) {
                t.cq[i] = op->ctrls[i];
                t.cm[i] = qubit_mask(op->ctrls[i]);
            }
            t.mat = (int)p.tmats.size();
            p.tmats.insert(p.tmats.end(), Ms.begin(), Ms.end());
        }
        p.tops.push_back(t);
    }
    p.members = (int)members.size();
}

void plan_tiles(qs_circuit *c, int T, int precision)
{
    const int N = c->num_qubits;
    const int n_ops = (int)c->ops.size();
    const int C = std::min(N, precision == QS_C64 ? 4 : 3);
    T = std::max(std::min(T, N), std::min(N, C + 3));
    std::vector<char> placed(n_ops, 0);
    const int lookahead = 512;
    for (int i = 0; i < n_ops; i++) {
        if (placed[i]) continue;
        const CircOp &first = c->ops[i];
        // controls beyond the 4 a tile operator carries, or gates of more
        // than 3 targets, run as passes of their own
        if (!absorbable(first) || first.ctrls.size() > 4) {
            placed[i] = 1;
            c->passes.push_back(single_pass(first));
            continue;
        }
        Echelon E;
        for (int b = 0; b < C; b++) E.add(1ULL << b);
        std::vector<const CircOp *> members;
        uint64_t blocked = 0;
        for (int j = i; j < n_ops && j < i + lookahead; j++) {
            if (placed[j]) continue;
            const CircOp &op = c->ops[j];
            const uint64_t s = support_mask(op);
            if (s & blocked) {
                blocked |= s;
                continue;
            }
            const std::vector<uint64_t> need = needed_vectors(op);
            if (absorbable(op) && op.ctrls.size() <= 4 && E.dim_with(need) <= T) {
                for (uint64_t x : need) E.add(x);
                members.push_back(&op);
                placed[j] = 1;
            } else {
                blocked |= s;
            }
            if (__builtin_popcountll(blocked) >= N) break;
        }
        Pass p{};
        encode_step(p, E, members);
        c->passes.push_back(std::move(p));
    }
}

size_t tile_pass_bytes(const Pass &p, int precision)
{
    const size_t ops = ((p.tops.size() * sizeof(TOp)) + 255) & ~size_t(255);
    return ops + p.tmats.size() * (precision == QS_C64 ? sizeof(float2) : sizeof(double2));
}

void pack_tile_pass(const Pass &p, int precision, void *out)
{
    unsigned char *o = (unsigned char *)out;
    std::memcpy(o, p.tops.data(), p.tops.size() * sizeof(TOp));
    unsigned char *m = o + (((p.tops.size() * sizeof(TOp)) + 255) & ~size_t(255));
    for (size_t i = 0; i < p.tmats.size(); i++) {
        if (precision == QS_C64)
            ((float2 *)m)[i] = make_float2((float)p.tmats[i].real(), (float)p.tmats[i].imag());
        else
            ((double2 *)m)[i] = make_double2(p.tmats[i].real(), p.tmats[i].imag());
    }
}

// ---- kernel -------------------------------------------------------------------------------
//
// EL = log2(tile entries per thread).  With EL fixed at compile time every
// per-operator loop is unrolled: a thread first loads all of its pairs or
// groups from LDS, then computes and stores them, so the LDS round trips of
// one operator overlap instead of running one after another.

struct TileArgs {
    int d;
    int nops;
    uint64_t w[kTileDimMax];
    InsertPlan plan;     // zeros at the pivots: spreads the tile number
    uint64_t num_tiles;
};

template <int NT>
__device__ __forceinline__ int spread_group(int g, const TOp &op)
{
#pragma unroll
    for (int i = 0; i < NT; i++) {
        const int lo = (1 << op.pos[i]) - 1;
        g = (g & lo) | ((g & ~lo) << 1);
    }
    return g;
}

template <int NT>
__device__ __forceinline__ int local_member(int cb, int l, const TOp &op)
{
#pragma unroll
    for (int i = 0; i < NT; i++)
        if ((l >> i) & 1) cb |= 1 << op.pos[i];
    return cb;
}

template <typename R, int NT, int EL>
__device__ void tile_dense(C2<R> *v, int d, const TOp &op, uint64_t base, const C2<R> *__restrict__ mat)
{
    constexpr int D = 1 << NT;
    constexpr int PER = (EL >= NT) ? (1 << (EL - NT)) : 1;   // groups per thread
    const int groups = 1 << (d - NT);
    C2<R> m[D * D];
#pragma unroll
    for (int k = 0; k < D * D; k++) m[k] = mat[k];
    int cb[PER];
    bool on[PER];
    C2<R> x[PER][D];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int g = threadIdx.x + u * blockDim.x;
        cb[u] = spread_group<NT>(g, op);
        bool ok = g < groups;
        for (int i = 0; i < op.nc; i++)
            ok &= (((base >> op.cq[i]) & 1ULL) ^ (uint64_t)(__popc(cb[u] & op.cm[i]) & 1)) != 0;
        on[u] = ok;
        if (ok) {
#pragma unroll
            for (int l = 0; l < D; l++) x[u][l] = v[local_member<NT>(cb[u], l, op)];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        if (!on[u]) continue;
#pragma unroll
        for (int j = 0; j < D; j++) {
            C2<R> acc = mk<R>(R(0), R(0));
#pragma unroll
            for (int l = 0; l < D; l++) cmac<R>(acc, m[j * D + l], x[u][l]);
            v[local_member<NT>(cb[u], j, op)] = acc;
        }
    }
}

template <typename R, int EL>
__device__ void tile_gadget(C2<R> *v, int d, const TOp &op, uint64_t base)
{
    const int sb = __popcll(base & op.yz) & 1;
    const R cs = (R)op.cs, cr = (R)op.cre, ci = (R)op.cim;
    if (op.flip == 0) {
        constexpr int PER = 1 << EL;
        const int T = 1 << d;
        C2<R> x[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int c = threadIdx.x + u * blockDim.x;
            if (c < T) x[u] = v[c];
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int c = threadIdx.x + u * blockDim.x;
            if (c < T) {
                const R s = ((sb ^ __popc((unsigned)c & op.yzm)) & 1) ? R(-1) : R(1);
                const C2<R> a = x[u];
                v[c] = mk<R>(cs * a.x + s * (cr * a.x - ci * a.y), cs * a.y + s * (cr * a.y + ci * a.x));
            }
        }
        return;
    }
    constexpr int PER = (EL >= 1) ? (1 << (EL - 1)) : 1;
    const int np = 1 << (d - 1);
    const int hb = 31 - __clz(op.flip);
    const int lo = (1 << hb) - 1;
    int c0[PER];
    C2<R> a0[PER], a1[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int p = threadIdx.x + u * blockDim.x;
        c0[u] = (p & lo) | ((p & ~lo) << 1);
        if (p < np) {
            a0[u] = v[c0[u]];
            a1[u] = v[c0[u] ^ (int)op.flip];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int p = threadIdx.x + u * blockDim.x;
        if (p >= np) continue;
        const int c1 = c0[u] ^ (int)op.flip;
        const R s0 = ((sb ^ __popc((unsigned)c0[u] & op.yzm)) & 1) ? R(-1) : R(1);
        const R s1 = ((sb ^ __popc((unsigned)c1 & op.yzm)) & 1) ? R(-1) : R(1);
        const C2<R> x0 = a0[u], x1 = a1[u];
        v[c0[u]] = mk<R>(cs * x0.x + s1 * (cr * x1.x - ci * x1.y), cs * x0.y + s1 * (cr * x1.y + ci * x1.x));
        v[c1] = mk<R>(cs * x1.x + s0 * (cr * x0.x - ci * x0.y), cs * x1.y + s0 * (cr * x0.y + ci * x0.x));
    }
}

template <typename R, int EL>
__global__ __launch_bounds__(1024) void k_tile_step(C2<R> *__restrict__ a, TileArgs ta, const TOp *__restrict__ tops,
                                                     const C2<R> *__restrict__ mats)
{
    extern __shared__ unsigned char lds_raw[];
    C2<R> *v = reinterpret_cast<C2<R> *>(lds_raw);
    constexpr int PER = 1 << EL;
    const int T = 1 << ta.d;
    const int lb = 31 - __clz(blockDim.x);   // block size is a power of two
    // coordinates c = threadIdx.x + blockDim.x u: the address is linear in c
    uint64_t xt = 0;
    for (int k = 0; k < lb && k < ta.d; k++)
        if ((threadIdx.x >> k) & 1) xt ^= ta.w[k];
    uint64_t xu[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        uint64_t x = xt;
        for (int k = lb; k < ta.d; k++)
            if ((u >> (k - lb)) & 1) x ^= ta.w[k];
        xu[u] = x;
    }
    for (uint64_t tile = blockIdx.x; tile < ta.num_tiles; tile += gridDim.x) {
        const uint64_t base = insert_zeros(tile, ta.plan);
#pragma unroll
        for (int u = 0; u < PER; u++)
            if ((int)threadIdx.x + (u << lb) < T) v[threadIdx.x + (u << lb)] = a[base ^ xu[u]];
        __syncthreads();
        for (int o = 0; o < ta.nops; o++) {
            const TOp &op = tops[o];
            if (op.kind == 1) {
                tile_gadget<R, EL>(v, ta.d, op, base);
            } else {
                const C2<R> *m = mats + op.mat;
                if (op.nt == 1) tile_dense<R, 1, EL>(v, ta.d, op, base, m);
                else if (op.nt == 2) tile_dense<R, 2, EL>(v, ta.d, op, base, m);
                else tile_dense<R, 3, EL>(v, ta.d, op, base, m);
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < PER; u++)
            if ((int)threadIdx.x + (u << lb) < T) a[base ^ xu[u]] = v[threadIdx.x + (u << lb)];
        __syncthreads();
    }
}

template <typename R>
static int launch_tile_r(qs_qureg *q, int el, unsigned grid, unsigned block, size_t lds, const TileArgs &ta,
                         const TOp *tops, const C2<R> *mats)
{
    C2<R> *amps = (C2<R> *)q->amps;
    switch (el) {
    case 0: hipLaunchKernelGGL((k_tile_step<R, 0>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    case 1: hipLaunchKernelGGL((k_tile_step<R, 1>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    case 2: hipLaunchKernelGGL((k_tile_step<R, 2>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    case 3: hipLaunchKernelGGL((k_tile_step<R, 3>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    case 4: hipLaunchKernelGGL((k_tile_step<R, 4>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    case 5: hipLaunchKernelGGL((k_tile_step<R, 5>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    default: hipLaunchKernelGGL((k_tile_step<R, 6>), dim3(grid), dim3(block), lds, q->stream, amps, ta, tops, mats); break;
    }
    QS_LAUNCH_CHECK();
    return QS_OK;
}

int launch_tile_pass(qs_qureg *q, const Pass &p, const void *dev)
{
    if (!dev) return fail(QS_E_PRECOND, "tile pass without device tables");
    TileArgs ta{};
    ta.d = p.tile_d;
    ta.nops = (int)p.tops.size();
    for (int k = 0; k < p.tile_d; k++) ta.w[k] = p.basis[k];
    ta.plan = make_insert_plan(p.pivots);
    ta.num_tiles = 1ULL << (q->index_bits - p.tile_d);
    const unsigned char *d = (const unsigned char *)dev;
    const unsigned char *mats = d + (((p.tops.size() * sizeof(TOp)) + 255) & ~size_t(255));
    const size_t ab = q->precision == QS_C64 ? sizeof(float2) : sizeof(double2);
    const size_t lds = ((size_t)1 << p.tile_d) * ab;
    // threads per block: 8 tile entries per thread (measured best), between
    // 64 and 1024 threads, unless QS_TILE_BLOCK overrides it
    int lb = std::min(10, std::max(6, p.tile_d - 3));
    if (const int forced = tile_block_size()) lb = 31 - __builtin_clz((unsigned)forced);
    while (p.tile_d - lb > 4 && lb < 10) lb++;
    const unsigned block = 1u << lb;
    const int el = std::max(0, p.tile_d - lb);
    const unsigned grid = grid_for(ta.num_tiles, 1, 0xFFFFFFFFull / block);
    if (q->precision == QS_C64)
        return launch_tile_r<float>(q, el, grid, block, lds, ta, (const TOp *)d, (const float2 *)mats);
    return launch_tile_r<double>(q, el, grid, block, lds, ta, (const TOp *)d, (const double2 *)mats);
}

}  // namespace qs
