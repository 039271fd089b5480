// Read-only passes over a state: Born probabilities, norm, trace, purity,
// Pauli-sum expectation values, inner products, and the partial trace.
// All sums accumulate in FP64: per thread, then across the wavefront by
// shuffles, across the block through LDS, and finally across blocks in a
// fixed order, so a result does not depend on scheduling.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>

namespace qs {



__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums (re, im) over the block; thread 0 receives the totals.
__device__ __forceinline__ void block_sum2(double &re, double &im)
{
    __shared__ double s_re[16], s_im[16];
    re = wave_sum(re);
    im = wave_sum(im);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_re[wave] = re; s_im[wave] = im; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double a = 0, b = 0;
        for (int w = 0; w < nw; w++) { a += s_re[w]; b += s_im[w]; }
        re = a;
        im = b;
    }
}

template <typename F>
__global__ __launch_bounds__(256) void k_reduce(F f, uint64_t n, double *__restrict__ partials)
{
    double re = 0.0, im = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // eight elements per round, so that their loads are in flight together
    // (the accumulations keep the index order: the sum stays deterministic)
    for (; i + 7 * stride < n; i += 8 * stride) {
#pragma unroll
        for (int k = 0; k < 8; k++) f(i + k * stride, re, im);
    }
    for (; i < n; i += stride) f(i, re, im);
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

// Fixed-order sum of `blocks` (re, im) partials into result[2*slot..].
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int blocks,
                                                   double *__restrict__ result, int slot)
{
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) {
        re += partials[2 * b];
        im += partials[2 * b + 1];
    }
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        result[2 * slot] = re;
        result[2 * slot + 1] = im;
    }
}

// ---- per-index contributions --------------------------------------------------------

template <typename R> struct SumSq {
    const C2<R> *a;
    __device__ void operator()(uint64_t i, double &re, double &) const
    {
        const C2<R> x = a[i];
        re += (double)x.x * x.x + (double)x.y * x.y;
    }
};

// Born rule on a statevector: amplitudes whose bit q equals b.
template <typename R> struct ProbSV {
    const C2<R> *a;
    uint64_t low;    // (1 << q) - 1
    uint64_t bit;    // b << q
    __device__ void operator()(uint64_t g, double &re, double &) const
    {
        const uint64_t i = (g & low) | ((g & ~low) << 1) | bit;
        const C2<R> x = a[i];
        re += (double)x.x * x.x + (double)x.y * x.y;
    }
};

// Diagonal of a density matrix: rho[k][k] sits at Choi index k (2^N + 1);
// optionally only k whose bit q equals b.
template <typename R> struct DiagDM {
    const C2<R> *a;
    uint64_t stride; // 2^N + 1
    uint64_t low, bit;
    int conditioned;
    __device__ void operator()(uint64_t g, double &re, double &im) const
    {
        const uint64_t k = conditioned ? ((g & low) | ((g & ~low) << 1) | bit) : g;
        const C2<R> x = a[k * stride];
        re += x.x;
        im += x.y;
    }
};

template <typename R> struct Inner {
    const C2<R> *a, *b;
    __device__ void operator()(uint64_t i, double &re, double &im) const
    {
        const C2<R> x = a[i], y = b[i];
        re += (double)x.x * y.x + (double)x.y * y.y;
        im += (double)x.x * y.y - (double)x.y * y.x;
    }
};

constexpr int kTermsPerLaunch = 24;

// Pauli terms sharing one flip mask: coefficient h_n eta_n (complex) and the
// sign mask yz_n of each.
struct TermGroup {
    int count;
    uint64_t yz[kTermsPerLaunch];
    double cre[kTermsPerLaunch], cim[kTermsPerLaunch];
};

__device__ __forceinline__ void group_coeff(const TermGroup &t, uint64_t x, double &re, double &im)
{
    re = 0.0;
    im = 0.0;
    for (int n = 0; n < t.count; n++) {
        const double s = (__popcll(x & t.yz[n]) & 1) ? -1.0 : 1.0;
        re = fma(s, t.cre[n], re);
        im = fma(s, t.cim[n], im);
    }
}

// <psi| sum_n h_n P_n |psi> over the pairs (i, j = i ^ xy), using
// (P psi)_i = beta_j a_j (Eq. "pauli_tensor_amp_update"), beta_x = eta (-1)^{popc(x & yz)}:
// contribution conj(a_i) c(j) a_j + conj(a_j) c(i) a_i with c(x) = sum_n h_n beta^{(n)}_x.
template <typename R> struct ExpecPairs {
    const C2<R> *a;
    uint64_t low, xy;
    TermGroup t;
    __device__ void operator()(uint64_t g, double &re, double &im) const
    {
        const uint64_t i = (g & low) | ((g & ~low) << 1);
        const uint64_t j = i ^ xy;
        const C2<R> ai = a[i], aj = a[j];
        double ci_re, ci_im, cj_re, cj_im;
        group_coeff(t, i, ci_re, ci_im);
        group_coeff(t, j, cj_re, cj_im);
        // conj(ai) * aj and conj(aj) * ai
        const double p_re = (double)ai.x * aj.x + (double)ai.y * aj.y;
        const double p_im = (double)ai.x * aj.y - (double)ai.y * aj.x;
        re += cj_re * p_re - cj_im * p_im + ci_re * p_re + ci_im * p_im;
        im += cj_re * p_im + cj_im * p_re - ci_re * p_im + ci_im * p_re;
    }
};

// Diagonal terms (no X or Y): sum_i |a_i|^2 sum_n h_n (-1)^{popc(i & z_n)}.
template <typename R> struct ExpecDiag {
    const C2<R> *a;
    TermGroup t;
    __device__ void operator()(uint64_t i, double &re, double &im) const
    {
        const C2<R> x = a[i];
        const double p = (double)x.x * x.x + (double)x.y * x.y;
        double c_re, c_im;
        group_coeff(t, i, c_re, c_im);
        re += c_re * p;
        im += c_im * p;
    }
};

// Tr(H rho) (Eq. "dens_expec_val_sum"): the Pauli tensor element
// P[l][k] is non-zero only for l = k ^ x, where it equals
// i^{#Y} (-1)^{popc(k & yz)}; so each term gathers the 2^N entries
// rho[k][k ^ x] = Choi[k + ((k ^ x) << N)] instead of visiting all 4^N.
struct DMTerms {
    int count;
    uint64_t x[kTermsPerLaunch], yz[kTermsPerLaunch];
    double cre[kTermsPerLaunch], cim[kTermsPerLaunch];   // h_n i^{#Y}
};

template <typename R> struct ExpecDM {
    const C2<R> *a;
    int N;
    DMTerms t;
    __device__ void operator()(uint64_t k, double &re, double &im) const
    {
        for (int n = 0; n < t.count; n++) {
            const C2<R> b = a[k + ((k ^ t.x[n]) << N)];
            const double s = (__popcll(k & t.yz[n]) & 1) ? -1.0 : 1.0;
            const double c_re = s * t.cre[n], c_im = s * t.cim[n];
            re += c_re * b.x - c_im * b.y;
            im += c_re * b.y + c_im * b.x;
        }
    }
};

// ---- Pauli sums on a statevector by tiles ----------------------------------------------
// <psi|P_n|psi> = sum_i conj(a_i) beta_j a_j, j = i ^ x_n (the same pairing as
// above).  A tile is a coset of V = span(e_0..e_{L-1}, w_0..w_{m-1}) where the
// w_k are an echelon basis of the flip masks of several terms: with the tile
// in LDS, each amplitude's partner j = i ^ x_n lies in the same tile for every
// one of them, so one read of the state serves them all.  Tile element c
// (a d-bit coordinate, d = L + m) sits at base ^ (c & (2^L - 1)) ^ xor of the
// w_k over the set bits L + k of c; in these coordinates x_n is a d-bit
// flip xc_n, and popc(j & yz_n) mod 2 is parity(base & yz_n) ^ parity(c_j & zc_n),
// zc_n bit k = parity(coordinate vector k & yz_n).
// For a Hermitian term the sum over i is real when parity(x_n & yz_n) = 0 and
// imaginary otherwise (partners i, j contribute conjugate products whose signs
// agree or differ), so a term accumulates one real number: the sum of
// (-1)^{popc(j & yz_n)} Re or Im of conj(a_i) a_j; the host applies h_n i^{#Y}.
// Block of 256 threads; thread t holds elements t + 256 u, u < E = 2^(d-8);
// d <= 11 and L = 4 (runs of 16 contiguous amplitudes), so m = 7 masks per span.
constexpr int kTileTerms = 8;
constexpr int kTileBlocks = 4096;   // most blocks of one launch

struct TileTermSet {
    int count;
    uint32_t kind;                  // bit n: term n sums Im (else Re)
    uint32_t xl[kTileTerms];        // coordinate flip, thread bits (c & 255)
    uint32_t xh[kTileTerms];        // coordinate flip, register bits (c >> 8)
    uint32_t zl[kTileTerms];        // coordinate sign mask, thread bits
    uint32_t zh[kTileTerms];        // coordinate sign mask, register bits
    uint64_t yz[kTileTerms];        // sign mask of the term (tile base parity)
    int pair[kTileTerms];           // half sums (E = 8): register bit 0-2 or 8 + thread bit; -1: full sum
};

struct TileSpan {
    InsertPlan plan;                // coset bases: zeros at the d pivot positions
    uint64_t coord[8];              // offsets of coordinates 0..7 (thread bits)
    uint64_t offu[8];               // offset of element 256 u
};

// One term's sum over the thread's elements of a tile, up to a sign that
// the caller applies: partner coordinate (t + 256 u) ^ xc, and
// (-1)^{popc((u ^ xh) & zh)} = (-1)^{popc(xh & zh)} (-1)^{popc(u & zh)}, the
// second factor summed as a fold over the register bits (one sign per bit).
// The partner of register u sits at byte tb + su, tb = (t ^ xl) times the
// element size (the thread's part) and su that of 256 (u ^ xh) (the same for
// every thread, a scalar): one vector add per LDS read.
// Each product Re or Im of conj(own) partner is formed in the precision of
// the amplitudes (complex64: FP32, whose tile in LDS is then half the bytes);
// every sum from there on is FP64.
template <bool IM, int E, typename R>
__device__ __forceinline__ double term_sum(const unsigned char *__restrict__ tile, const C2<R> (&own)[E], uint32_t tb,
                                           uint32_t xh, uint32_t zh)
{
    double p[E];
#pragma unroll
    for (int u = 0; u < E; u++) {
        const uint32_t su = __builtin_amdgcn_readfirstlane(((uint32_t)u ^ xh) * 256u * (uint32_t)sizeof(C2<R>));
        const C2<R> v = *(const C2<R> *)(tile + (tb + su));
        const R w = IM ? own[u].x * v.y - own[u].y * v.x : own[u].x * v.x + own[u].y * v.y;
        p[u] = (double)w;
    }
#pragma unroll
    for (int h = E / 2; h >= 1; h >>= 1) {
        const double sg = (zh & (uint32_t)h) ? -1.0 : 1.0;
#pragma unroll
        for (int u = 0; u < h; u++) p[u] = fma(sg, p[u + h], p[u]);
    }
    return p[0];
}

// Half sums (tiles of 8 registers).  For a Hermitian Pauli string the two
// products of a pair (i, j = i ^ x) agree once the term's sign is applied:
// Re (or Im) of conj(a_i) a_j (-1)^{j.z} equals that of conj(a_j) a_i
// (-1)^{i.z}, because (-1)^{x.z} is +1 exactly for the terms that sum Re.
// So each pair is taken once, from the element whose pairing bit is clear,
// and the caller doubles the sum.
// Register pairing (x flips register bit RB, the lowest of xh): the
// registers u with bit RB clear, partners u ^ xh; the fold's signs come from
// the other two register bits.
template <bool IM, int RB, typename R>
__device__ __forceinline__ double term_half_reg(const unsigned char *__restrict__ tile, const C2<R> (&own)[8],
                                                uint32_t tb, uint32_t xh, uint32_t zh)
{
    constexpr int ub0 = RB == 0 ? 1 : 0, ub1 = RB == 2 ? 1 : 2;   // register bits of k's bits 0 and 1
    double p[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int u = ((k >> RB) << (RB + 1)) | (k & ((1 << RB) - 1));
        const uint32_t su = __builtin_amdgcn_readfirstlane(((uint32_t)u ^ xh) * 256u * (uint32_t)sizeof(C2<R>));
        const C2<R> v = *(const C2<R> *)(tile + (tb + su));
        const R w = IM ? own[u].x * v.y - own[u].y * v.x : own[u].x * v.x + own[u].y * v.y;
        p[k] = (double)w;
    }
    const double s1 = ((zh >> ub1) & 1u) ? -1.0 : 1.0, s0 = ((zh >> ub0) & 1u) ? -1.0 : 1.0;
    p[0] = fma(s1, p[2], p[0]);
    p[1] = fma(s1, p[3], p[1]);
    return fma(s0, p[1], p[0]);
}

// Thread pairing (x flips thread bits only): thread t takes the registers u
// whose bit 2 equals bit b of t (b a flipped thread bit), its own values read
// back from LDS: ob, pb = byte offsets of (t, 4 q) and (t ^ xl, 4 q), q that
// bit of t; the sign of register bit 2 is the caller's.
template <bool IM, typename R>
__device__ __forceinline__ double term_half_thr(const unsigned char *__restrict__ tile, uint32_t ob, uint32_t pb,
                                                uint32_t zh)
{
    double p[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t off = (uint32_t)k * 256u * (uint32_t)sizeof(C2<R>);
        const C2<R> o = *(const C2<R> *)(tile + (ob + off));
        const C2<R> v = *(const C2<R> *)(tile + (pb + off));
        const R w = IM ? o.x * v.y - o.y * v.x : o.x * v.x + o.y * v.y;
        p[k] = (double)w;
    }
    const double s1 = ((zh >> 1) & 1u) ? -1.0 : 1.0, s0 = (zh & 1u) ? -1.0 : 1.0;
    p[0] = fma(s1, p[2], p[0]);
    p[1] = fma(s1, p[3], p[1]);
    return fma(s0, p[1], p[0]);
}

// One term over the thread's elements of the tile with its pairing (pr:
// TileTermSet::pair); extra: a sign bit the caller adds to the term's
// parity; twice: the sum counts each pair once.
template <bool IM, int E, typename R>
__device__ __forceinline__ double term_any(const unsigned char *__restrict__ tile, const C2<R> (&own)[E], uint32_t t,
                                           uint32_t tp, uint32_t xh, uint32_t zh, int pr, uint32_t &extra,
                                           bool &twice)
{
    constexpr uint32_t sz = (uint32_t)sizeof(C2<R>);
    if constexpr (E == 8) {
        if (pr >= 8) {
            const uint32_t q = (t >> (pr - 8)) & 1u;
            extra = q & (zh >> 2);
            twice = true;
            return term_half_thr<IM, R>(tile, (t + 1024u * q) * sz, (tp + 1024u * q) * sz, zh);
        }
        if (pr >= 0) {
            twice = true;
            if (pr == 0) return term_half_reg<IM, 0, R>(tile, own, tp * sz, xh, zh);
            if (pr == 1) return term_half_reg<IM, 1, R>(tile, own, tp * sz, xh, zh);
            return term_half_reg<IM, 2, R>(tile, own, tp * sz, xh, zh);
        }
    }
    return term_sum<IM, E, R>(tile, own, tp * sz, xh, zh);
}

template <typename R, int E>
__global__ __launch_bounds__(256) void k_expec_tiles(const C2<R> *__restrict__ a, uint64_t num_tiles, TileSpan sp,
                                                     TileTermSet ts, double *__restrict__ partials)
{
    __shared__ C2<R> tile[256 * E];
    __shared__ double red[kTileTerms][4];
    const uint32_t t = threadIdx.x;
    uint64_t toff = 0;
#pragma unroll
    for (int k = 0; k < 8; k++)
        if ((t >> k) & 1) toff ^= sp.coord[k];
    double acc[kTileTerms];
#pragma unroll
    for (int n = 0; n < kTileTerms; n++) acc[n] = 0.0;

    uint64_t g = blockIdx.x;
    C2<R> x[E];
    if (g < num_tiles) {
        const uint64_t b0 = insert_zeros(g, sp.plan);
#pragma unroll
        for (int u = 0; u < E; u++) x[u] = a[b0 ^ sp.offu[u] ^ toff];
    }
    for (; g < num_tiles; g += gridDim.x) {
        const uint64_t base = insert_zeros(g, sp.plan);
        C2<R> own[E];
#pragma unroll
        for (int u = 0; u < E; u++) own[u] = x[u];
        __syncthreads();    // the previous tile's reads are done
#pragma unroll
        for (int u = 0; u < E; u++) tile[t + 256 * u] = own[u];
        __syncthreads();
        // the next tile's loads go out before the sums
        const uint64_t next = g + gridDim.x;
#pragma unroll
        for (int u = 0; u < E; u++) x[u] = mk<R>(R(0), R(0));
        if (next < num_tiles) {
            const uint64_t nb = insert_zeros(next, sp.plan);
#pragma unroll
            for (int u = 0; u < E; u++) x[u] = a[nb ^ sp.offu[u] ^ toff];
        }
        // t made opaque per tile: the partner addresses of every (term, u)
        // are loop invariants that would otherwise stay live in registers
        uint32_t tv = t;
        asm volatile("" : "+v"(tv));
#pragma unroll
        for (int n = 0; n < kTileTerms; n++) {
            if (n < ts.count) {
                const uint32_t tp = tv ^ ts.xl[n];
                uint32_t zh = ts.zh[n];      // likewise for the fold signs
                asm volatile("" : "+s"(zh));
                const unsigned char *tl = reinterpret_cast<const unsigned char *>(tile);
                uint32_t extra = 0;
                bool twice = false;
                const double s =
                    ((ts.kind >> n) & 1)
                        ? term_any<true, E, R>(tl, own, tv, tp, ts.xh[n], zh, ts.pair[n], extra, twice)
                        : term_any<false, E, R>(tl, own, tv, tp, ts.xh[n], zh, ts.pair[n], extra, twice);
                const uint32_t par = (uint32_t)__popcll(base & ts.yz[n]) + (uint32_t)__popc(ts.xh[n] & ts.zh[n]) +
                                     (uint32_t)__popc(tp & ts.zl[n]) + extra;
                const double w = twice ? 2.0 : 1.0;
                acc[n] = fma((par & 1) ? -w : w, s, acc[n]);
            }
        }
    }
    // per term: wave sums, then the four waves in order
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int n = 0; n < kTileTerms; n++) {
        if (n < ts.count) {
            const double v = wave_sum(acc[n]);
            if (lane == 0) red[n][wave] = v;
        }
    }
    __syncthreads();
    if ((int)t < ts.count)
        partials[(size_t)t * gridDim.x + blockIdx.x] = ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
}

// Term n's block partials summed in block order into result[slot0 + n].
__global__ __launch_bounds__(256) void k_finalize_terms(const double *__restrict__ partials, int blocks,
                                                         double *__restrict__ result, int slot0)
{
    double re = 0.0, im = 0.0;
    const double *p = partials + (size_t)blockIdx.x * blocks;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) re += p[b];
    block_sum2(re, im);
    if (threadIdx.x == 0) result[slot0 + blockIdx.x] = re;
}

// ---- purity: Tr(rho^2) = sum_{k,l} rho[k][l] rho[l][k] ---------------------------------
// Tiles of TS x TS entries: tile (kb, lb) with kb <= lb is read with k
// fastest, its mirror with l fastest, the mirror goes through LDS so each
// thread multiplies matching entries; off-diagonal tiles count twice.
constexpr int kTile = 32;

template <typename R>
__global__ __launch_bounds__(256) void k_purity(const C2<R> *__restrict__ a, int N, int TS, uint64_t tiles_per_dim,
                                                 uint64_t num_pairs, double *__restrict__ partials)
{
    __shared__ double2 mirror[kTile][kTile + 1];
    const uint64_t d = 1ULL << N;
    double re = 0.0, im = 0.0;
    for (uint64_t p = blockIdx.x; p < num_pairs; p += gridDim.x) {
        uint64_t lb = (uint64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
        while (lb * (lb + 1) / 2 > p) lb--;
        while ((lb + 1) * (lb + 2) / 2 <= p) lb++;
        const uint64_t kb = p - lb * (lb + 1) / 2;
        const double w = (kb == lb) ? 1.0 : 2.0;
        __syncthreads();
        // mirror[kk][ll] = rho[l][k] = Choi[l + k d], loaded with ll fastest
        for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
            const int ll = e % TS, kk = e / TS;
            const C2<R> v = a[(lb * TS + ll) + (kb * TS + kk) * d];
            mirror[kk][ll] = make_double2(v.x, v.y);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < TS * TS; e += blockDim.x) {
            const int kk = e % TS, ll = e / TS;
            const C2<R> v = a[(kb * TS + kk) + (lb * TS + ll) * d];
            const double2 m = mirror[kk][ll];
            re += w * ((double)v.x * m.x - (double)v.y * m.y);
            im += w * ((double)v.x * m.y + (double)v.y * m.x);
        }
    }
    (void)tiles_per_dim;
    block_sum2(re, im);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = re;
        partials[2 * blockIdx.x + 1] = im;
    }
}

// ---- partial trace (Eq. "partial_trace_reduced_amp_def") -------------------------------
//
// The entries that the trace reads are those whose bit t + N equals bit t for
// every traced qubit t.  They are indexed by L, the Choi index with the bits
// t + N removed (2N - n bits): the address of L is L with zeros spliced in at
// the positions t + N, each then set to the bit t of L.  The low N bits of the
// address are those of L, so a wavefront whose lanes take the 6 lowest bits of
// L reads 64 consecutive entries.  Lanes that differ only in traced bits below
// 6 belong to the same output and are summed by shuffles; the traced bits from
// 6 up are the thread's loop (split over S waves of the block, whose partial
// sums meet in LDS, when the loop is long and the threads few).  Removing the
// traced positions from L gives the output index (kept row bits, then kept
// column bits, each in qubit order).
struct PTracePlan {
    InsertPlan top;       // zeros at the positions t + N (address space)
    InsertPlan hi;        // zeros at the traced positions >= 6 (L space): spreads the thread number
    uint64_t lo_mask;     // traced positions < 6 (lane bits)
    uint64_t slice_mask;  // the lowest log2(S) traced positions >= 6: which part of the loop a wave takes
    uint64_t loop_mask;   // the other traced positions >= 6: the loop of every thread
    uint64_t num_threads; // 2^(2N - n - n_hi)
    int N;
    int slices;           // S, waves per lane group
    int groups;           // lane groups of 64 threads per block
};

template <typename R>
__global__ __launch_bounds__(1024) void k_partial_trace(const C2<R> *__restrict__ in, C2<R> *__restrict__ out,
                                                        PTracePlan p)
{
    __shared__ double s_part[16][64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slice = wave % p.slices, group = wave / p.slices;
    const uint64_t T = ((uint64_t)blockIdx.x * p.groups + group) * 64 + lane;
    const bool live = T < p.num_threads;
    double re = 0.0, im = 0.0;
    if (live) {
        const uint64_t L = insert_zeros(T, p.hi);
        uint64_t base = insert_zeros(L, p.top);
        uint64_t lo = L & p.lo_mask;
        base |= lo << p.N;
        // this wave's fixed slice bits: the slice number deposited in slice_mask
        uint64_t sl = 0;
        {
            uint64_t m = p.slice_mask;
            for (int b = 0; m; b++, m &= m - 1)
                if ((slice >> b) & 1) sl |= m & (~m + 1);
        }
        base |= sl | (sl << p.N);
        // every subset s of loop_mask in increasing order: s' = ((s | ~M) + 1) & M
        uint64_t s = 0;
        const uint64_t M = p.loop_mask;
        const uint64_t count = 1ULL << __popcll(M);
        uint64_t j = 0;
        // eight loads in flight before their sums (same order of additions)
        for (; j + 8 <= count; j += 8) {
            C2<R> x[8];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                x[k] = in[base | s | (s << p.N)];
                s = ((s | ~M) + 1) & M;
            }
#pragma unroll
            for (int k = 0; k < 8; k++) {
                re += (double)x[k].x;
                im += (double)x[k].y;
            }
        }
        for (; j < count; j++) {
            const C2<R> x = in[base | s | (s << p.N)];
            re += (double)x.x;
            im += (double)x.y;
            s = ((s | ~M) + 1) & M;
        }
    }
    if (p.slices > 1) {
        s_part[wave][lane][0] = re;
        s_part[wave][lane][1] = im;
        __syncthreads();
        if (slice == 0) {
            re = 0.0;
            im = 0.0;
            for (int k = 0; k < p.slices; k++) {
                re += s_part[wave + k][lane][0];
                im += s_part[wave + k][lane][1];
            }
        }
    }
    if (slice != 0) return;   // wave-uniform
    // sum over the traced lane bits, lowest first
#pragma unroll
    for (int b = 0; b < 6; b++)
        if ((p.lo_mask >> b) & 1) {
            re += __shfl_xor(re, 1 << b, 64);
            im += __shfl_xor(im, 1 << b, 64);
        }
    if (!live || (lane & p.lo_mask)) return;
    uint64_t o = 0;
    int w = 0;
    for (int b = 0; b < 6; b++)
        if (!((p.lo_mask >> b) & 1)) o |= (uint64_t)((lane >> b) & 1) << w++;
    o |= (T >> 6) << w;
    out[o] = mk<R>((R)re, (R)im);
}

// ---- host drivers ----------------------------------------------------------------------

template <typename F>
static int run_reduce(qs_qureg *q, const F &f, uint64_t n, int slot)
{
    const int blocks = (int)grid_for(n, 256, kReduceBlocks);
    hipLaunchKernelGGL(k_reduce<F>, dim3(blocks), dim3(256), 0, q->stream, f, n, q->d_partials);
    QS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, q->stream, (const double *)q->d_partials, blocks,
                       q->d_result, slot);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

// Copies result slots [0, nslots) back and waits.
static int fetch(qs_qureg *q, int nslots)
{
    QS_HIP(hipMemcpyAsync(q->h_result, q->d_result, sizeof(double) * 2 * nslots, hipMemcpyDeviceToHost, q->stream));
    QS_HIP(hipStreamSynchronize(q->stream));
    return QS_OK;
}

int finish_reduction(qs_qureg *q, int blocks, int slot, double *out)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, q->stream, (const double *)q->d_partials, blocks,
                       q->d_result, slot);
    QS_LAUNCH_CHECK();
    int rc = fetch(q, slot + 1);
    if (rc != QS_OK) return rc;
    out[0] = q->h_result[2 * slot];
    out[1] = q->h_result[2 * slot + 1];
    return QS_OK;
}

template <typename R>
static int sum_sq(qs_qureg *q, double *out)
{
    int rc = run_reduce(q, SumSq<R>{(const C2<R> *)q->amps}, q->num_amps, 0);
    if (rc == QS_OK) rc = fetch(q, 1);
    if (rc == QS_OK) *out = q->h_result[0];
    return rc;
}

template <typename R>
static int diag_dm(qs_qureg *q, int qubit, int outcome, double *re, double *im)
{
    DiagDM<R> f{(const C2<R> *)q->amps, (1ULL << q->num_qubits) + 1ULL, 0, 0, 0};
    uint64_t n = 1ULL << q->num_qubits;
    if (qubit >= 0) {
        f.low = (1ULL << qubit) - 1ULL;
        f.bit = (uint64_t)outcome << qubit;
        f.conditioned = 1;
        n >>= 1;
    }
    int rc = run_reduce(q, f, n, 0);
    if (rc == QS_OK) rc = fetch(q, 1);
    if (rc != QS_OK) return rc;
    *re = q->h_result[0];
    if (im) *im = q->h_result[1];
    return QS_OK;
}

template <typename R>
static int prob_sv(qs_qureg *q, int qubit, int outcome, double *out)
{
    ProbSV<R> f{(const C2<R> *)q->amps, (1ULL << qubit) - 1ULL, (uint64_t)outcome << qubit};
    int rc = run_reduce(q, f, q->num_amps >> 1, 0);
    if (rc == QS_OK) rc = fetch(q, 1);
    if (rc == QS_OK) *out = q->h_result[0];
    return rc;
}

template <typename R>
static int expec_sv(qs_qureg *q, const int *codes, const double *coeffs, int T, double *re, double *im)
{
    const int N = q->num_qubits;
    // group the terms by their flip mask
    std::map<uint64_t, std::vector<int>> groups;
    std::vector<uint64_t> yzs(T);
    std::vector<cd> cs(T);
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    for (int t = 0; t < T; t++) {
        uint64_t xy = 0, yz = 0;
        int ny = 0;
        for (int k = 0; k < N; k++) {
            const int c = codes[(size_t)t * N + k];
            if (c < 0 || c > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
            if (c == 1 || c == 2) xy |= 1ULL << k;
            if (c == 2 || c == 3) yz |= 1ULL << k;
            if (c == 2) ny++;
        }
        groups[xy].push_back(t);
        yzs[t] = yz;
        cs[t] = coeffs[t] * eta[ny & 3];
    }
    double acc_re = 0.0, acc_im = 0.0;
    int slot = 0;
    auto flush = [&]() -> int {
        if (slot == 0) return QS_OK;
        int rc = fetch(q, slot);
        if (rc != QS_OK) return rc;
        for (int s = 0; s < slot; s++) {
            acc_re += q->h_result[2 * s];
            acc_im += q->h_result[2 * s + 1];
        }
        slot = 0;
        return QS_OK;
    };
    for (auto &kv : groups) {
        const uint64_t xy = kv.first;
        const std::vector<int> &ts = kv.second;
        for (size_t b = 0; b < ts.size(); b += kTermsPerLaunch) {
            TermGroup g{};
            g.count = (int)std::min<size_t>(kTermsPerLaunch, ts.size() - b);
            for (int n = 0; n < g.count; n++) {
                g.yz[n] = yzs[ts[b + n]];
                g.cre[n] = cs[ts[b + n]].real();
                g.cim[n] = cs[ts[b + n]].imag();
            }
            int rc;
            if (xy == 0) {
                rc = run_reduce(q, ExpecDiag<R>{(const C2<R> *)q->amps, g}, q->num_amps, slot);
            } else {
                const int hb = 63 - __builtin_clzll(xy);   // see k_gadget_pairs
                rc = run_reduce(q, ExpecPairs<R>{(const C2<R> *)q->amps, (1ULL << hb) - 1ULL, xy, g},
                                q->num_amps >> 1, slot);
            }
            if (rc != QS_OK) return rc;
            if (++slot == kResultSlots / 2) {
                rc = flush();
                if (rc != QS_OK) return rc;
            }
        }
    }
    int rc = flush();
    if (rc != QS_OK) return rc;
    *re = acc_re;
    *im = acc_im;
    return QS_OK;
}

// Blocks of one k_expec_tiles<R, E> launch: twice as many as stay resident
// (at most kTileBlocks), each walking tiles by a fixed stride.  On the
// 20-term sum over 28 qubits, against 1024 blocks: complex64 1.60 against
// 1.76 ms per call (as many as stay resident: 1.65 ms), complex128 2.41
// against 2.66 ms; runs of consecutive tiles per block were no faster.
template <typename R>
static int expec_tile_blocks(int E, int device)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(device, E);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    hipError_t e1;
    if (E == 1) e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_expec_tiles<R, 1>, 256, 0);
    else if (E == 2) e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_expec_tiles<R, 2>, 256, 0);
    else if (E == 4) e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_expec_tiles<R, 4>, 256, 0);
    else e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_expec_tiles<R, 8>, 256, 0);
    const hipError_t e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    int blocks = 1024;
    if (e1 == hipSuccess && e2 == hipSuccess && per_cu >= 1 && cus >= 1) blocks = std::min(kTileBlocks, 2 * per_cu * cus);
    else (void)hipGetLastError();
    cache.emplace(key, blocks);
    return blocks;
}

template <typename R>
static void launch_expec_tiles(int E, int blocks, hipStream_t st, const C2<R> *amps, uint64_t num_tiles,
                               const TileSpan &sp, const TileTermSet &ts, double *partials)
{
    if (E == 1) hipLaunchKernelGGL((k_expec_tiles<R, 1>), dim3(blocks), dim3(256), 0, st, amps, num_tiles, sp, ts, partials);
    else if (E == 2) hipLaunchKernelGGL((k_expec_tiles<R, 2>), dim3(blocks), dim3(256), 0, st, amps, num_tiles, sp, ts, partials);
    else if (E == 4) hipLaunchKernelGGL((k_expec_tiles<R, 4>), dim3(blocks), dim3(256), 0, st, amps, num_tiles, sp, ts, partials);
    else hipLaunchKernelGGL((k_expec_tiles<R, 8>), dim3(blocks), dim3(256), 0, st, amps, num_tiles, sp, ts, partials);
}

// Tiled Pauli sum for N >= 8: spans of L low qubits plus up to d - L flip
// masks (greedy, first fit over the distinct masks in ascending order), each
// span's terms in launches of up to kTileTerms.
template <typename R>
static int expec_sv_tiles(qs_qureg *q, const int *codes, const double *coeffs, int T, double *re, double *im)
{
    const int N = q->num_qubits;
    const int d = std::min(N, 11);
    const int L = 4;
    const int m = d - L;
    const uint64_t lowmask = (1ULL << L) - 1ULL;
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    std::vector<uint64_t> xs(T), yzs(T);
    std::vector<cd> cs(T);
    std::map<uint64_t, std::vector<int>> by_mask;
    for (int t = 0; t < T; t++) {
        uint64_t xy = 0, yz = 0;
        int ny = 0;
        for (int k = 0; k < N; k++) {
            const int c = codes[(size_t)t * N + k];
            if (c < 0 || c > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
            if (c == 1 || c == 2) xy |= 1ULL << k;
            if (c == 2 || c == 3) yz |= 1ULL << k;
            if (c == 2) ny++;
        }
        xs[t] = xy;
        yzs[t] = yz;
        cs[t] = coeffs[t] * eta[ny & 3];
        by_mask[xy].push_back(t);
    }
    std::vector<uint64_t> pending;
    for (auto &kv : by_mask) pending.push_back(kv.first);

    double acc_re = 0.0, acc_im = 0.0;
    int slot = 0;
    std::vector<int> slot_term;
    auto flush = [&]() -> int {
        if (slot == 0) return QS_OK;
        QS_HIP(hipMemcpyAsync(q->h_result, q->d_result, sizeof(double) * slot, hipMemcpyDeviceToHost, q->stream));
        QS_HIP(hipStreamSynchronize(q->stream));
        for (int s = 0; s < slot; s++) {
            const int t = slot_term[s];
            const double v = q->h_result[s];
            if (__builtin_popcountll(xs[t] & yzs[t]) & 1) {     // i v
                acc_re -= cs[t].imag() * v;
                acc_im += cs[t].real() * v;
            } else {
                acc_re += cs[t].real() * v;
                acc_im += cs[t].imag() * v;
            }
        }
        slot = 0;
        slot_term.clear();
        return QS_OK;
    };

    while (!pending.empty()) {
        // reduced echelon basis of the high parts (pivot = highest bit)
        std::vector<uint64_t> basis;
        std::vector<uint64_t> chosen, rest;
        for (uint64_t x : pending) {
            uint64_t r = x & ~lowmask;
            for (uint64_t b : basis)
                if (r >> (63 - __builtin_clzll(b)) & 1) r ^= b;
            if (r == 0) {
                chosen.push_back(x);
            } else if ((int)basis.size() < m) {
                const int p = 63 - __builtin_clzll(r);
                for (uint64_t &b : basis)
                    if ((b >> p) & 1) b ^= r;
                basis.push_back(r);
                chosen.push_back(x);
            } else {
                rest.push_back(x);
            }
        }
        pending.swap(rest);
        // remaining coordinates L + k: pad with unit vectors on free qubits
        std::vector<int> pivots;
        for (uint64_t b : basis) pivots.push_back(63 - __builtin_clzll(b));
        // (N >= d leaves enough free columns); clearing column b from the
        // others keeps every pivot column in one basis vector only
        for (int b = L; (int)basis.size() < m && b < N; b++) {
            if (std::find(pivots.begin(), pivots.end(), b) != pivots.end()) continue;
            for (uint64_t &v : basis) v &= ~(1ULL << b);
            basis.push_back(1ULL << b);
            pivots.push_back(b);
        }
        std::vector<int> order(m);
        for (int k = 0; k < m; k++) order[k] = k;
        std::sort(order.begin(), order.end(), [&](int i, int j) { return pivots[i] < pivots[j]; });
        std::vector<uint64_t> coord(d);
        std::vector<int> pos;
        for (int k = 0; k < L; k++) { coord[k] = 1ULL << k; pos.push_back(k); }
        for (int k = 0; k < m; k++) { coord[L + k] = basis[order[k]]; pos.push_back(pivots[order[k]]); }
        std::sort(pos.begin(), pos.end());
        TileSpan sp{};
        sp.plan.n = d;
        for (int k = 0; k < d; k++) sp.plan.low[k] = (1ULL << pos[k]) - 1ULL;
        for (int k = 0; k < 8; k++) sp.coord[k] = coord[k];
        const int E = 1 << (d - 8);
        for (int u = 0; u < E; u++) {
            uint64_t o = 0;
            for (int k = 0; k < d - 8; k++)
                if ((u >> k) & 1) o ^= coord[8 + k];
            sp.offu[u] = o;
        }
        // coordinates of a flip mask and of a sign mask
        auto flip_coord = [&](uint64_t x) {
            uint32_t c = (uint32_t)(x & lowmask);
            for (int k = 0; k < m; k++)
                if ((x >> pivots[order[k]]) & 1) c |= 1u << (L + k);
            return c;
        };
        auto sign_coord = [&](uint64_t yz) {
            uint32_t c = 0;
            for (int k = 0; k < d; k++)
                if (__builtin_popcountll(coord[k] & yz) & 1) c |= 1u << k;
            return c;
        };
        std::vector<int> terms;
        for (uint64_t x : chosen)
            for (int t : by_mask[x]) terms.push_back(t);
        const uint64_t num_tiles = 1ULL << (N - d);
        const int blocks = (int)std::min<uint64_t>(num_tiles, (uint64_t)expec_tile_blocks<R>(E, q->device));
        for (size_t b0 = 0; b0 < terms.size(); b0 += kTileTerms) {
            TileTermSet ts{};
            ts.count = (int)std::min<size_t>(kTileTerms, terms.size() - b0);
            if (slot + ts.count > kResultSlots) {
                int rc = flush();
                if (rc != QS_OK) return rc;
            }
            for (int n = 0; n < ts.count; n++) {
                const int t = terms[b0 + n];
                const uint32_t xc = flip_coord(xs[t]), zc = sign_coord(yzs[t]);
                ts.xl[n] = xc & 255u;
                ts.xh[n] = xc >> 8;
                ts.zl[n] = zc & 255u;
                ts.zh[n] = zc >> 8;
                ts.yz[n] = yzs[t];
                // pairing of the half sums: the lowest flipped register bit,
                // else the highest flipped thread bit (tiles of 8 registers)
                ts.pair[n] = -1;
                if (E == 8 && ts.xh[n]) ts.pair[n] = __builtin_ctz(ts.xh[n]);
                else if (E == 8 && ts.xl[n]) ts.pair[n] = 8 + (31 - __builtin_clz(ts.xl[n]));
                if (__builtin_popcountll(xs[t] & yzs[t]) & 1) ts.kind |= 1u << n;
                slot_term.push_back(t);
            }
            launch_expec_tiles<R>(E, blocks, q->stream, (const C2<R> *)q->amps, num_tiles, sp, ts, q->d_partials);
            QS_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_finalize_terms, dim3(ts.count), dim3(256), 0, q->stream,
                               (const double *)q->d_partials, blocks, q->d_result, slot);
            QS_LAUNCH_CHECK();
            slot += ts.count;
        }
    }
    int rc = flush();
    if (rc != QS_OK) return rc;
    *re = acc_re;
    *im = acc_im;
    return QS_OK;
}

template <typename R>
static int expec_dm(qs_qureg *q, const int *codes, const double *coeffs, int T, double *re, double *im)
{
    const int N = q->num_qubits;
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    double acc_re = 0.0, acc_im = 0.0;
    for (int b = 0; b < T; b += kTermsPerLaunch) {
        DMTerms g{};
        g.count = std::min(kTermsPerLaunch, T - b);
        for (int n = 0; n < g.count; n++) {
            uint64_t x = 0, yz = 0;
            int ny = 0;
            for (int k = 0; k < N; k++) {
                const int c = codes[(size_t)(b + n) * N + k];
                if (c < 0 || c > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
                if (c == 1 || c == 2) x |= 1ULL << k;
                if (c == 2 || c == 3) yz |= 1ULL << k;
                if (c == 2) ny++;
            }
            const cd c = coeffs[b + n] * eta[ny & 3];
            g.x[n] = x;
            g.yz[n] = yz;
            g.cre[n] = c.real();
            g.cim[n] = c.imag();
        }
        int rc = run_reduce(q, ExpecDM<R>{(const C2<R> *)q->amps, N, g}, 1ULL << N, 0);
        if (rc == QS_OK) rc = fetch(q, 1);
        if (rc != QS_OK) return rc;
        acc_re += q->h_result[0];
        acc_im += q->h_result[1];
    }
    *re = acc_re;
    *im = acc_im;
    return QS_OK;
}

template <typename R>
static int purity(qs_qureg *q, double *re, double *im)
{
    const int N = q->num_qubits;
    const uint64_t d = 1ULL << N;
    const int TS = (int)std::min<uint64_t>(d, kTile);
    const uint64_t T = d / TS;
    const uint64_t pairs = T * (T + 1) / 2;
    const int blocks = (int)std::min<uint64_t>(pairs, kReduceBlocks);
    hipLaunchKernelGGL(k_purity<R>, dim3(blocks), dim3(256), 0, q->stream, (const C2<R> *)q->amps, N, TS, T, pairs,
                       q->d_partials);
    QS_LAUNCH_CHECK();
    double out[2];
    int rc = finish_reduction(q, blocks, 0, out);
    if (rc != QS_OK) return rc;
    *re = out[0];
    if (im) *im = out[1];
    return QS_OK;
}

template <typename R>
static int partial_trace(const qs_qureg *in, const std::vector<int> &t, qs_qureg *out)
{
    const int N = in->num_qubits, n = (int)t.size();
    PTracePlan p{};
    std::vector<int> top, hi;
    for (int x : t) {
        top.push_back(x + N);
        if (x >= 6) hi.push_back(x); else p.lo_mask |= 1ULL << x;
    }
    std::sort(hi.begin(), hi.end());
    p.top = make_insert_plan(top);
    p.hi = make_insert_plan(hi);
    p.N = N;
    const int n_hi = (int)hi.size();
    p.num_threads = 1ULL << (2 * N - n - n_hi);
    // split the loop over up to 16 waves while the threads are few
    int slices = 1, sbits = 0;
    while (slices < 16 && sbits < n_hi && p.num_threads * (uint64_t)slices < (1ULL << 17)) {
        slices *= 2;
        sbits++;
    }
    for (int k = 0; k < n_hi; k++) {
        if (k < sbits) p.slice_mask |= 1ULL << hi[k];
        else p.loop_mask |= 1ULL << hi[k];
    }
    p.slices = slices;
    const int waves = std::max(4, slices);
    p.groups = waves / slices;
    const uint64_t lane_groups = (p.num_threads + 63) / 64;
    const uint64_t blocks = (lane_groups + p.groups - 1) / p.groups;
    if (blocks > 0xFFFFFFFFull / (64ull * waves)) return fail(QS_E_ARG, "partial trace too large for one launch");
    hipLaunchKernelGGL(k_partial_trace<R>, dim3((unsigned)blocks), dim3(64 * waves), 0, in->stream,
                       (const C2<R> *)in->amps, (C2<R> *)out->amps, p);
    QS_LAUNCH_CHECK();
    (void)out;
    return QS_OK;
}

// Pauli sum on a statevector (tiles for N >= 8, else pairs per flip mask)
// or a density matrix.  Scratch: q->d_partials (at most kExpecPartials
// doubles: 2 per reduction block, or one per tile block and term) and
// q->d_result (kResultSlots doubles); no staging of matrices.
static_assert(kExpecPartials >= 2 * (size_t)kReduceBlocks, "reduction partials exceed the bound");
static_assert(kExpecPartials >= (size_t)kTileBlocks * kTileTerms, "tile partials exceed the bound");
int expec_pauli_sum(qs_qureg *q, const int *paulis, const double *coeffs, int num_terms, double *out_re,
                           double *out_im)
{
    if (num_terms < 0 || (num_terms > 0 && (!paulis || !coeffs))) return fail(QS_E_ARG, "bad Pauli sum");
    double re = 0.0, im = 0.0;
    int rc = QS_OK;
    if (num_terms > 0) {
        if (q->is_density)
            rc = q->precision == QS_C64 ? expec_dm<float>(q, paulis, coeffs, num_terms, &re, &im)
                                        : expec_dm<double>(q, paulis, coeffs, num_terms, &re, &im);
        else if (q->num_qubits >= 8)
            rc = q->precision == QS_C64 ? expec_sv_tiles<float>(q, paulis, coeffs, num_terms, &re, &im)
                                        : expec_sv_tiles<double>(q, paulis, coeffs, num_terms, &re, &im);
        else
            rc = q->precision == QS_C64 ? expec_sv<float>(q, paulis, coeffs, num_terms, &re, &im)
                                        : expec_sv<double>(q, paulis, coeffs, num_terms, &re, &im);
    }
    if (rc != QS_OK) return rc;
    if (out_re) *out_re = re;
    if (out_im) *out_im = im;
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int qs_calc_total_prob(const qs_qureg *cq, double *out)
{
    qs_qureg *q = const_cast<qs_qureg *>(cq);
    if (!q || !out) return fail(QS_E_ARG, "null argument");
    if (q->is_density)
        return q->precision == QS_C64 ? diag_dm<float>(q, -1, 0, out, nullptr) : diag_dm<double>(q, -1, 0, out, nullptr);
    return q->precision == QS_C64 ? sum_sq<float>(q, out) : sum_sq<double>(q, out);
}

int qs_calc_prob_of_outcome(const qs_qureg *cq, int qubit, int outcome, double *out)
{
    qs_qureg *q = const_cast<qs_qureg *>(cq);
    if (!q || !out) return fail(QS_E_ARG, "null argument");
    if (qubit < 0 || qubit >= q->num_qubits) return fail(QS_E_ARG, "qubit out of range");
    if (outcome != 0 && outcome != 1) return fail(QS_E_ARG, "outcome must be 0 or 1");
    if (q->is_density)
        return q->precision == QS_C64 ? diag_dm<float>(q, qubit, outcome, out, nullptr)
                                      : diag_dm<double>(q, qubit, outcome, out, nullptr);
    return q->precision == QS_C64 ? prob_sv<float>(q, qubit, outcome, out) : prob_sv<double>(q, qubit, outcome, out);
}

int qs_calc_trace(const qs_qureg *cq, double *out_re, double *out_im)
{
    qs_qureg *q = const_cast<qs_qureg *>(cq);
    if (!q || !out_re) return fail(QS_E_ARG, "null argument");
    if (!q->is_density) return fail(QS_E_PRECOND, "trace is defined here for density matrices");
    return q->precision == QS_C64 ? diag_dm<float>(q, -1, 0, out_re, out_im) : diag_dm<double>(q, -1, 0, out_re, out_im);
}

int qs_calc_purity(const qs_qureg *cq, double *out_re, double *out_im)
{
    qs_qureg *q = const_cast<qs_qureg *>(cq);
    if (!q || !out_re) return fail(QS_E_ARG, "null argument");
    if (!q->is_density) return fail(QS_E_PRECOND, "purity is computed for density matrices");
    return q->precision == QS_C64 ? purity<float>(q, out_re, out_im) : purity<double>(q, out_re, out_im);
}

int qs_calc_expec_pauli_sum(const qs_qureg *cq, const int *paulis, const double *coeffs, int num_terms,
                            double *out_re, double *out_im)
{
    qs_qureg *q = const_cast<qs_qureg *>(cq);
    if (!q) return fail(QS_E_ARG, "null qureg");
    return expec_pauli_sum(q, paulis, coeffs, num_terms, out_re, out_im);
}

int qs_calc_inner_product(const qs_qureg *ca, const qs_qureg *cb, double *out_re, double *out_im)
{
    qs_qureg *a = const_cast<qs_qureg *>(ca);
    qs_qureg *b = const_cast<qs_qureg *>(cb);
    if (!a || !b) return fail(QS_E_ARG, "null qureg");
    if (a->is_density || b->is_density) return fail(QS_E_PRECOND, "inner products of statevectors only");
    if (a->num_qubits != b->num_qubits) return fail(QS_E_ARG, "qubit counts differ");
    if (a->precision != b->precision) return fail(QS_E_TYPE, "precisions differ");
    if (a->stream != b->stream) QS_HIP(hipStreamSynchronize(b->stream));
    int rc = a->precision == QS_C64
                 ? run_reduce(a, Inner<float>{(const float2 *)a->amps, (const float2 *)b->amps}, a->num_amps, 0)
                 : run_reduce(a, Inner<double>{(const double2 *)a->amps, (const double2 *)b->amps}, a->num_amps, 0);
    if (rc == QS_OK) rc = fetch(a, 1);
    if (rc != QS_OK) return rc;
    if (out_re) *out_re = a->h_result[0];
    if (out_im) *out_im = a->h_result[1];
    return QS_OK;
}

int qs_calc_partial_trace(const qs_qureg *in, const int *targs, int num_targs, qs_qureg *out)
{
    if (!in || !out) return fail(QS_E_ARG, "null qureg");
    if (!in->is_density || !out->is_density) return fail(QS_E_PRECOND, "partial trace needs density matrices");
    if (in->precision != out->precision) return fail(QS_E_TYPE, "precisions differ");
    if (num_targs < 1 || num_targs >= in->num_qubits || !targs)
        return fail(QS_E_ARG, "trace out between 1 and N-1 qubits");
    if (num_targs > kMaxInsert) return fail(QS_E_ARG, "too many traced qubits");
    if (out->num_qubits != in->num_qubits - num_targs)
        return fail(QS_E_ARG, "output must have N - n qubits");
    if (in->amps == out->amps) return fail(QS_E_ARG, "input and output must not alias");
    std::string why;
    if (!valid_qubits(targs, num_targs, in->num_qubits, why)) return fail(QS_E_ARG, why);
    // out's pending work must finish before in's stream overwrites it, and
    // out's later work must follow the trace
    if (out->stream != in->stream) QS_HIP(hipStreamSynchronize(out->stream));
    std::vector<int> t(targs, targs + num_targs);
    int rc = in->precision == QS_C64 ? partial_trace<float>(in, t, out) : partial_trace<double>(in, t, out);
    if (rc != QS_OK) return rc;
    if (out->stream != in->stream) QS_HIP(hipStreamSynchronize(in->stream));
    return QS_OK;
}

}  // extern "C"
