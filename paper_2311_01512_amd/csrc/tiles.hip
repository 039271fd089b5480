// Tile engine for recorded circuits.
//
// A step owns a subspace span(W) of the index space (GF(2) vectors, at most
// T dimensions) that always contains the unit vectors of the lowest C
// qubits, so each tile is read in runs of at least 2^C consecutive
// amplitudes (a full 128-byte line).  A dense gate fits a step when the unit
// vectors of its targets lie in span(W); a Pauli gadget fits when its X/Y
// flip mask does, whatever its weight, since the gadget only pairs i with
// i ^ x.  Each tile (coset base ^ span(W)) is read once from HBM into
// registers, every operator of the step is applied, and the tile is written
// back: one HBM pass for the whole step.  Operators join a step only if they
// commute with every operator they jump over (no shared qubit), so the
// circuit's order holds.
//
// Inside a step the operators run in phases.  In a phase each thread holds
// kRegs tile elements whose coordinates form a coset of a kRegBits-dimensional
// register subspace that contains the target unit vectors and flip vectors
// of all the phase's operators, so every operator only mixes registers of
// one thread: no LDS traffic and no barrier per operator.  Between phases
// the tile moves through LDS once to the next layout.
#include "circuit.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

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

// Gates of up to 3 targets run on registers; 4-target gates only on the
// matrix cores (complex64 tiles of at least 2^9 amplitudes).
static bool absorbable(const CircOp &op, bool mfma)
{
    return op.gadget || op.targs.size() <= 3 || (mfma && op.targs.size() == 4);
}

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

// ---- phases -----------------------------------------------------------------------------

// Register basis of a phase in tile coordinates: the unit vectors of the
// register targets first, then the gadget flips reduced against what is
// there, then (if pad) unit vectors of the highest free coordinates up to
// kRegBits.  A vector's pivot is its highest set bit outside `excl` (the
// lane coordinates of an MFMA phase); every vector has no free bit above its
// pivot, so the set is independent of itself and of the unit vectors of all
// other coordinates.  Returns the number of vectors, or -1 when a target
// is excluded or a flip lies in span(r) + span(excl) but not in span(r).
static int reg_basis(const std::vector<int> &units, const std::vector<uint32_t> &flips, uint32_t excl, int d,
                     bool pad, std::vector<uint32_t> &r, std::vector<int> &piv)
{
    r.clear();
    piv.clear();
    auto reduce = [&](uint32_t x) {
        std::vector<size_t> order(r.size());
        for (size_t j = 0; j < r.size(); j++) order[j] = j;
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return piv[a] > piv[b]; });
        for (size_t j : order)
            if ((x >> piv[j]) & 1u) x ^= r[j];
        return x;
    };
    for (int c : units) {
        if ((excl >> c) & 1u) return -1;
        if (std::find(piv.begin(), piv.end(), c) != piv.end()) continue;
        r.push_back(1u << c);
        piv.push_back(c);
    }
    for (uint32_t f : flips) {
        const uint32_t x = reduce(f);
        if (!x) continue;
        const uint32_t free_bits = x & ~excl;
        if (!free_bits) return -1;
        r.push_back(x);
        piv.push_back(31 - __builtin_clz(free_bits));
    }
    if (pad)
        for (int c = d - 1; c >= 0 && (int)r.size() < kRegBits; c--) {
            if (((excl >> c) & 1u) || std::find(piv.begin(), piv.end(), c) != piv.end()) continue;
            r.push_back(1u << c);
            piv.push_back(c);
        }
    return (int)r.size();
}

// A phase under construction: lane coordinates of its MFMA operators (or
// none), register target coordinates, gadget flips.
struct PhaseBuild {
    int c4 = -1, c5 = -1;
    std::vector<int> units;
    std::vector<uint32_t> flips;
    uint32_t excl() const { return c4 < 0 ? 0u : ((1u << c4) | (1u << c5)); }
    bool fits() const
    {
        std::vector<uint32_t> r;
        std::vector<int> piv;
        const int n = reg_basis(units, flips, excl(), 32, false, r, piv);
        return n >= 0 && n <= kRegBits;
    }
};

// Real coefficients of a k-target gate (k = 2, 3, 4) for v_mfma_f32_16x16x4f32.
// Lane L of the wavefront holds, in register u, the element whose lane
// coordinates c4, c5 carry g ^ h(u) (g = L / 16; h(u) = the bits of rho[u] at
// c4, c5) in group L % 16, and further members in registers for the register-
// target bits rho; member index i = (g ^ h) + 4 rho.  K-step s feeds the real
// (s even) or imaginary part of register rho = s / 2; output block b,
// register i of lane group g' receives component o = 4 b + i, i.e. the real
// (o even) or imaginary part of member (g' ^ h) + 4 (o / 2).  Lane L supplies
// A[L % 16][L / 16] of each (b, s).  Layout: [h][lane][b][s], NB * KS floats
// per lane, four variants h = 0..3.
static void mfma_coeffs(const std::vector<cd> &G, int k, std::vector<cd> &out)
{
    const int R = 1 << (k - 2), KS = 2 * R, NB = R >= 2 ? R / 2 : 1;
    const int D = 1 << k;
    std::vector<float> a((size_t)4 * 64 * NB * KS, 0.f);
    for (int h = 0; h < 4; h++)
        for (int L = 0; L < 64; L++) {
            const int m = L % 16, gp = m / 4, i = m % 4, g = L / 16;
            for (int b = 0; b < NB; b++)
                for (int s = 0; s < KS; s++) {
                    const int o = 4 * b + i;
                    float v = 0.f;
                    if (o < 2 * R) {
                        const int iout = (gp ^ h) + 4 * (o / 2), iin = (g ^ h) + 4 * (s / 2);
                        const cd z = G[(size_t)iout * D + iin];
                        const int po = o % 2, pi = s % 2;
                        v = (float)(po == pi ? z.real() : (po ? z.imag() : -z.imag()));
                    }
                    a[((size_t)h * 64 + L) * NB * KS + b * KS + s] = v;
                }
        }
    for (size_t j = 0; j < a.size(); j += 2) out.push_back(cd(a[j], a[j + 1]));
}

// Operators of a finished step in the step's coordinates, grouped in phases.
static void encode_step(Pass &p, const Echelon &E, const std::vector<const CircOp *> &members, bool mfma)
{
    p.tile = true;
    p.gadget = false;
    p.basis.clear();
    p.pivots.clear();
    for (auto &kv : E.by_pivot) {
        p.pivots.push_back(kv.first);
        p.basis.push_back(kv.second);
    }
    const int d = (int)p.basis.size();
    p.tile_d = d;
    const int lb = d - kRegBits;
    mfma = mfma && lb >= 6;   // lane bits 4 and 5 must exist, every wave full
    auto coord_of_pivot = [&](int b) {
        return (int)(std::find(p.pivots.begin(), p.pivots.end(), b) - p.pivots.begin());
    };
    auto qubit_mask = [&](int b) {
        uint32_t m = 0;
        for (int k = 0; k < d; k++)
            if ((p.basis[k] >> b) & 1ULL) m |= 1u << k;
        return m;
    };
    auto flip_of = [&](uint64_t x) {
        uint32_t f = 0;
        for (int k = 0; k < d; k++)
            if ((x >> p.pivots[k]) & 1ULL) f |= 1u << k;
        return f;
    };
    auto addr_of = [&](uint32_t c) {
        uint64_t a = 0;
        for (int k = 0; k < d; k++)
            if ((c >> k) & 1u) a ^= p.basis[k];
        return a;
    };
    // coordinate needs of each member: target unit vectors or the gadget flip
    struct Need {
        std::vector<int> units;
        uint32_t flip;
        uint64_t x, yz;
        int ny;
    };
    std::vector<Need> needs(members.size());
    for (size_t i = 0; i < members.size(); i++) {
        const CircOp *op = members[i];
        Need &n = needs[i];
        n.flip = 0;
        n.x = n.yz = 0;
        n.ny = 0;
        if (op->gadget) {
            for (size_t k = 0; k < op->targs.size(); k++) {
                const int c = op->paulis[k];
                const uint64_t b = 1ULL << op->targs[k];
                if (c == 1 || c == 2) n.x |= b;
                if (c == 2 || c == 3) n.yz |= b;
                if (c == 2) n.ny++;
            }
            n.flip = flip_of(n.x);
        } else {
            for (int t : op->targs) n.units.push_back(coord_of_pivot(t));
        }
    }
    // Fits member m into phase B: a gadget by its flip; a dense gate of <= 3
    // targets in registers; a gate of 3-4 targets that does not fit there on
    // the matrix cores (two targets on the lane coordinates, the rest in
    // registers).  Gates of 2-3 targets measured no faster on the matrix cores
    // (a 2-target gate as a real 8 x 8 product fills half of the 16 x 16
    // tile), so the matrix cores are what lets 4-target gates (two-qubit
    // superoperators) join a step.  Returns the mode (0 registers, 1 MFMA) or -1.
    auto try_fit = [&](PhaseBuild &B, size_t m) {
        const Need &n = needs[m];
        const CircOp *op = members[m];
        if (op->gadget) {
            PhaseBuild T = B;
            if (n.flip) T.flips.push_back(n.flip);
            if (!T.fits()) return -1;
            B = T;
            return 0;
        }
        const int nt = (int)n.units.size();
        if (nt <= 3) {
            PhaseBuild T = B;
            T.units.insert(T.units.end(), n.units.begin(), n.units.end());
            if (T.fits()) {
                B = T;
                return 0;
            }
        }
        if (!mfma || nt < 3) return -1;
        std::vector<int> us = n.units;
        std::sort(us.begin(), us.end());
        PhaseBuild T = B;
        std::vector<int> rest;
        if (T.c4 < 0) {
            T.c4 = us[0];
            T.c5 = us[1];
            rest.assign(us.begin() + 2, us.end());
        } else {
            if (std::find(us.begin(), us.end(), T.c4) == us.end() || std::find(us.begin(), us.end(), T.c5) == us.end())
                return -1;
            for (int c : us)
                if (c != T.c4 && c != T.c5) rest.push_back(c);
        }
        T.units.insert(T.units.end(), rest.begin(), rest.end());
        if (!T.fits()) return -1;
        B = T;
        return 1;
    };
    const cd eta[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
    p.phases.clear();
    p.rops.clear();
    p.tmats.clear();
    // Gadgets run as cos(theta) (1 + i tan(theta) eta P): the real factors
    // cos(theta) of the step multiply every amplitude alike, so they are
    // collected in `scale` and folded into one uncontrolled matrix of the step
    // (or applied by a scaling operator at its end).  A factored gadget can
    // grow an amplitude by up to 1 + |tan(theta)|; gadgets with |cos| < 1/64
    // keep the unfactored form, as do all once the step's growth bound would
    // pass 2^64.
    double scale = 1.0, growth = 1.0;
    std::vector<std::pair<size_t, size_t>> mat_range;   // tmats entries of each operator
    // A phase takes, in order, every remaining member that fits it and shares
    // no qubit with a remaining member it jumps over.
    std::vector<size_t> remaining(members.size());
    for (size_t m = 0; m < members.size(); m++) remaining[m] = m;
    while (!remaining.empty()) {
        PhaseBuild B;
        std::vector<size_t> chosen, rest;
        std::vector<int> mode;
        uint64_t blocked = 0;
        for (size_t m : remaining) {
            const uint64_t s = support_mask(*members[m]);
            int md = -1;
            if (!(s & blocked)) md = try_fit(B, m);
            if (md >= 0) {
                chosen.push_back(m);
                mode.push_back(md);
            } else {
                blocked |= s;
                rest.push_back(m);
            }
        }
        remaining.swap(rest);
        std::vector<uint32_t> r;
        std::vector<int> pj;
        reg_basis(B.units, B.flips, B.excl(), d, true, r, pj);
        RPhase ph{};
        uint32_t taken = 0;   // pivots and lane coordinates: not deposited from t in order
        for (int b = 0; b < kRegBits; b++) taken |= 1u << pj[b];
        std::vector<int> ins(pj.begin(), pj.end());
        ph.c4 = ph.c5 = -1;
        if (B.c4 >= 0) {
            ph.c4 = B.c4;
            ph.c5 = B.c5;
            ins.push_back(B.c4);
            ins.push_back(B.c5);
            taken |= B.excl();
        }
        std::sort(ins.begin(), ins.end());
        ph.nlo = (int)ins.size();
        for (size_t b = 0; b < ins.size(); b++) ph.lo[b] = (1u << ins[b]) - 1u;
        for (int u = 0; u < kRegs; u++) {
            uint32_t c = 0;
            for (int b = 0; b < kRegBits; b++)
                if ((u >> b) & 1) c ^= r[b];
            ph.rho[u] = c;
            ph.yaddr[u] = addr_of(c);
        }
        // thread bit k -> coordinate: bits 4 and 5 to the lane coordinates of
        // an MFMA phase, the others in order to the free coordinates
        for (int k = 0, c = 0; k < lb; k++) {
            if (B.c4 >= 0 && (k == 4 || k == 5)) {
                ph.taddr[k] = p.basis[k == 4 ? B.c4 : B.c5];
                continue;
            }
            while ((taken >> c) & 1u) c++;
            ph.taddr[k] = p.basis[c];
            c++;
        }
        ph.first_op = (int)p.rops.size();
        ph.num_ops = (int)chosen.size();
        auto reg_bit_of_unit = [&](int coord) {
            for (int b = 0; b < kRegBits; b++)
                if (r[b] == (1u << coord)) return b;
            return -1;
        };
        for (size_t ci = 0; ci < chosen.size(); ci++) {
            const size_t m = chosen[ci];
            const CircOp *op = members[m];
            const Need &n = needs[m];
            const size_t mat0 = p.tmats.size();
            ROp ro{};
            if (op->gadget) {
                uint32_t f = n.flip, fu = 0;
                while (f) {
                    const uint32_t fb = f & ~B.excl();
                    const int hb = 31 - __builtin_clz(fb);
                    int b = 0;
                    while (b < kRegBits && pj[b] != hb) b++;
                    f ^= r[b];
                    fu |= 1u << b;
                }
                ro.yz = n.yz;
                uint32_t ym = 0;
                for (int b = 0; b < 64; b++)
                    if ((n.yz >> b) & 1ULL) ym ^= qubit_mask(b);
                ro.yzm = ym;
                for (int b = 0; b < kRegBits; b++) ro.gy |= (uint32_t)(__builtin_popcount(r[b] & ym) & 1) << b;
                const cd c = cd(0, std::sin(op->theta)) * eta[n.ny & 3];
                const double partner = (__builtin_popcountll(n.x & n.yz) & 1) ? -1.0 : 1.0;
                const double cs = std::cos(op->theta);
                const double tn = std::fabs(std::tan(op->theta));
                if (std::fabs(cs) >= 1.0 / 64 && growth * (1.0 + tn) <= 0x1p64) {
                    // c / cos(theta) = i tan(theta) eta: imaginary for an even
                    // number of Y (codes 24+), real for an odd one (40+)
                    const bool im = (n.ny & 1) == 0;
                    const double k = (im ? c.imag() : c.real()) / cs;
                    ro.code = (im ? 24 : 40) + (int)fu;
                    ro.cs = 1.0;
                    ro.cre = k;
                    ro.cim = 0.0;
                    ro.pre = partner * k;
                    ro.pim = 0.0;
                    scale *= cs;
                    growth *= 1.0 + tn;
                } else {
                    ro.code = 8 + (int)fu;
                    ro.cs = cs;
                    ro.cre = c.real();
                    ro.cim = c.imag();
                    ro.pre = partner * c.real();
                    ro.pim = partner * c.imag();
                }
                ro.fcs = (float)ro.cs;
                ro.fcre = (float)ro.cre;
                ro.fcim = (float)ro.cim;
                ro.fpre = (float)ro.pre;
                ro.fpim = (float)ro.pim;
            } else {
                ro.nc = (int)op->ctrls.size();
                for (int q = 0; q < ro.nc; q++) {
                    ro.cq[q] = op->ctrls[q];
                    ro.cm[q] = qubit_mask(op->ctrls[q]);
                }
                for (int u = 0; u < kRegs; u++) {
                    uint64_t nib = 0;
                    for (int q = 0; q < ro.nc; q++) nib |= (uint64_t)(__builtin_popcount(ph.rho[u] & ro.cm[q]) & 1) << q;
                    ro.qtab |= nib << (4 * u);
                }
                // sort keys: matrix bit order of the kernel
                std::vector<int> keys, sorted;
                uint32_t um = 0;
                if (mode[ci] == 1) {
                    for (int c : n.units) {
                        if (c == B.c4) keys.push_back(-2);
                        else if (c == B.c5) keys.push_back(-1);
                        else {
                            keys.push_back(reg_bit_of_unit(c));
                            um |= 1u << keys.back();
                        }
                    }
                    std::vector<cd> Ms = permute_to_sorted(op->M, keys, sorted);
                    ro.code = 32 + (int)um;
                    ro.mat = (int)p.tmats.size();
                    for (int u = 0; u < kRegs; u++)
                        ro.hsel |= (((ph.rho[u] >> B.c4) & 1u) | (((ph.rho[u] >> B.c5) & 1u) << 1)) << (2 * u);
                    mfma_coeffs(Ms, (int)n.units.size(), p.tmats);
                } else {
                    for (int c : n.units) {
                        keys.push_back(reg_bit_of_unit(c));
                        um |= 1u << keys.back();
                    }
                    std::vector<cd> Ms = permute_to_sorted(op->M, keys, sorted);
                    ro.code = (int)um + (ro.nc > 0 ? 16 : 0);
                    // uncontrolled 1-2 target gates that only couple members
                    // i and i ^ s (diagonal: s = 0), e.g. one-qubit channels
                    // as superoperators: the sparse form
                    const int D = 1 << n.units.size();
                    if (ro.nc == 0 && D <= 4) {
                        uint32_t xs = 0;   // set of r ^ c with a nonzero entry
                        for (int rr = 0; rr < D; rr++)
                            for (int cc = 0; cc < D; cc++)
                                if (Ms[(size_t)rr * D + cc] != cd(0, 0)) xs |= 1u << (rr ^ cc);
                        xs &= ~1u;
                        if (xs == 0 || (D == 4 && (xs & (xs - 1)) == 0))
                            ro.code = 64 + 4 * (int)um + (xs ? __builtin_ctz(xs) : 0);
                    }
                    ro.mat = (int)p.tmats.size();
                    p.tmats.insert(p.tmats.end(), Ms.begin(), Ms.end());
                }
            }
            p.rops.push_back(ro);
            mat_range.emplace_back(mat0, p.tmats.size());
        }
        p.phases.push_back(ph);
    }
    if (scale != 1.0) {
        // an uncontrolled dense, sparse or matrix-core operator takes the
        // factor in its matrix (every such form is linear in the matrix)
        // (FP64 register matrices first; matrix-core coefficients are FP32)
        bool folded = false;
        for (int pass = 0; pass < 2 && !folded; pass++)
            for (size_t i = 0; i < p.rops.size() && !folded; i++) {
                const ROp &ro = p.rops[i];
                const bool reg = (ro.code >= 1 && ro.code <= 7) || ro.code >= 64;
                const bool core = ro.code >= 32 && ro.code <= 38 && ro.nc == 0;
                if ((pass == 0 ? reg : core) && mat_range[i].second > mat_range[i].first) {
                    for (size_t k = mat_range[i].first; k < mat_range[i].second; k++) p.tmats[k] *= scale;
                    folded = true;
                }
            }
        if (!folded) {
            ROp ro{};
            ro.code = 16;
            ro.cs = scale;
            ro.fcs = (float)scale;
            p.rops.push_back(ro);
            p.phases.back().num_ops++;
        }
    }
    p.members = (int)members.size();
}

void plan_tiles(qs_circuit *c, int T, int precision)
{
    const int N = c->index_bits;
    const int n_ops = (int)c->ops.size();
    const int C = std::min(N, tile_low_qubits(precision));
    T = std::min(T, N);
    // dense gates of 2-4 targets on the FP32 matrix cores (complex64 only)
    const bool mfma = precision == QS_C64 && T >= kRegBits + 6;
    const int lookahead = 512;
    std::vector<char> placed(n_ops, 0);
    for (int i = 0; i < n_ops; i++) {
        if (placed[i]) continue;
        const CircOp &first = c->ops[i];
        // registers need a tile of more than kRegBits dimensions; controls
        // beyond the 4 a tile operator carries, or gates of more than 3
        // targets, run as passes of their own
        if (T <= kRegBits || !absorbable(first, mfma) || first.ctrls.size() > 4) {
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
            if (absorbable(op, mfma) && op.ctrls.size() <= 4 && E.dim_with(need) <= T) {
                for (uint64_t x : need) E.add(x);
                members.push_back(&op);
                placed[j] = 1;
            } else {
                blocked |= s;
            }
            if (__builtin_popcountll(blocked) >= N) break;
        }
        // fill the tile to T dimensions with the lowest free qubits: longer
        // contiguous runs, fewer and larger tiles
        for (int b = C; b < N && E.dim() < T; b++) E.add(1ULL << b);
        Pass p{};
        encode_step(p, E, members, mfma);
        c->passes.push_back(std::move(p));
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t tile_pass_bytes(const Pass &p, int precision)
{
    return align256(p.phases.size() * sizeof(RPhase)) + align256(p.rops.size() * sizeof(ROp)) +
           p.tmats.size() * (precision == QS_C64 ? sizeof(float2) : sizeof(double2));
}

void pack_tile_pass(const Pass &p, int precision, void *out)
{
    unsigned char *o = (unsigned char *)out;
    std::memcpy(o, p.phases.data(), p.phases.size() * sizeof(RPhase));
    o += align256(p.phases.size() * sizeof(RPhase));
    std::memcpy(o, p.rops.data(), p.rops.size() * sizeof(ROp));
    o += align256(p.rops.size() * sizeof(ROp));
    for (size_t i = 0; i < p.tmats.size(); i++) {
        if (precision == QS_C64)
            ((float2 *)o)[i] = make_float2((float)p.tmats[i].real(), (float)p.tmats[i].imag());
        else
            ((double2 *)o)[i] = make_double2(p.tmats[i].real(), p.tmats[i].imag());
    }
}

// ---- kernel -------------------------------------------------------------------------------

struct TileArgs {
    int d;
    int nph;
    InsertPlan plan;     // zeros at the tile's pivots: spreads the tile number
    uint64_t num_tiles;
};

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
    if constexpr (std::is_same<R, float>::value) {
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
    if constexpr (std::is_same<R, float>::value) {
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
    if constexpr (std::is_same<R, float>::value) f = op.fcs;
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
template <int RM>
__device__ __forceinline__ void mfma_dense(float2 (&x)[kRegs], const ROp &op, uint32_t tau, uint64_t base,
                                           const float2 *__restrict__ mats)
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    constexpr int R = 1 << popcount_c(RM), KS = 2 * R, NB = R >= 2 ? R / 2 : 1;
    const float *A0 = reinterpret_cast<const float *>(mats + op.mat) + (threadIdx.x & 63u) * (NB * KS);
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
            for (int s = 0; s < KS; s++) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[blk * KS + s], b[s], acc, 0, 0, 0);
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
    constexpr bool f32 = std::is_same<R, float>::value;
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

// Persistent blocks of 2^(d - kRegBits) threads, each walking tiles
// blockIdx.x + k gridDim.x.  A tile is read from HBM straight into the first
// phase's layout and written from the last one's; the next tile's loads are
// issued before the current tile's operators run, so they are in flight
// during the arithmetic (barriers here wait for LDS only).  Tiles are
// disjoint, so the early read sees no write of this launch.
template <typename R>
__global__ __launch_bounds__(1024) void k_tile_step(C2<R> *__restrict__ a, TileArgs ta, const RPhase *__restrict__ ph,
                                                     const ROp *__restrict__ ops, const C2<R> *__restrict__ mats)
{
    extern __shared__ unsigned char lds_raw[];
    const uint32_t t = threadIdx.x;
    const int lb = ta.d - kRegBits;
    const RPhase &first = ph[0];
    const RPhase &last = ph[ta.nph - 1];
    const uint64_t xg = thread_offset(t, lb, first);
    const uint64_t xs = thread_offset(t, lb, last);
    uint64_t tile = blockIdx.x;
    if (tile >= ta.num_tiles) return;
    C2<R> x[kRegs];
    {
        const uint64_t b0 = insert_zeros(tile, ta.plan);
#pragma unroll
        for (int u = 0; u < kRegs; u++) x[u] = a[b0 ^ xg ^ first.yaddr[u]];
        // the first tile is waited for here, so that inside the loop the
        // only memory wait is for the prefetch, never for earlier stores
#pragma unroll
        for (int u = 0; u < kRegs; u++) asm volatile("" ::"v"(x[u].x), "v"(x[u].y));
    }
    for (; tile < ta.num_tiles; tile += gridDim.x) {
        const uint64_t base = insert_zeros(tile, ta.plan);
        const uint64_t next = tile + gridDim.x;
        const bool more = next < ta.num_tiles;
        C2<R> nx[kRegs];
        if (more) {
            const uint64_t nb = insert_zeros(next, ta.plan);
#pragma unroll
            for (int u = 0; u < kRegs; u++) nx[u] = a[nb ^ xg ^ first.yaddr[u]];
        }
        uint32_t tau = tau_of(t, first);
        for (int p = 0; p < ta.nph; p++) {
            const RPhase &P = ph[p];
            if (p > 0) {
                const RPhase &Q = ph[p - 1];
                const uint32_t tn = tau_of(t, P);
                constexpr int sh = sizeof(C2<R>) == 8 ? 3 : 4;
                const uint32_t ob = tau << sh, nb = tn << sh;
                __syncthreads();   // earlier reads of the LDS tile are done
#pragma unroll
                for (int u = 0; u < kRegs; u++) *(C2<R> *)(lds_raw + (ob ^ (Q.rho[u] << sh))) = x[u];
                __syncthreads();
#pragma unroll
                for (int u = 0; u < kRegs; u++) x[u] = *(const C2<R> *)(lds_raw + (nb ^ (P.rho[u] << sh)));
                tau = tn;
            }
            const int end = P.first_op + P.num_ops;
            for (int o = P.first_op; o < end; o++) apply_reg_op<R>(x, ops[o], tau, base, mats);
        }
#pragma unroll
        for (int u = 0; u < kRegs; u++) a[base ^ xs ^ last.yaddr[u]] = x[u];
        if (more) {
#pragma unroll
            for (int u = 0; u < kRegs; u++) x[u] = nx[u];
        }
    }
}

int launch_tile_pass(qs_qureg *q, const Pass &p, const void *dev)
{
    if (!dev) return fail(QS_E_PRECOND, "tile pass without device tables");
    if (p.phases.empty()) return QS_OK;
    if (p.tile_d <= kRegBits || p.tile_d > kTileDimMax) return fail(QS_E_ARG, "tile dimension out of range");
    TileArgs ta{};
    ta.d = p.tile_d;
    ta.nph = (int)p.phases.size();
    ta.plan = make_insert_plan(p.pivots);
    ta.num_tiles = 1ULL << (q->index_bits - p.tile_d);
    const unsigned char *d = (const unsigned char *)dev;
    const RPhase *ph = (const RPhase *)d;
    const ROp *ops = (const ROp *)(d + align256(p.phases.size() * sizeof(RPhase)));
    const unsigned char *mats = (const unsigned char *)ops + align256(p.rops.size() * sizeof(ROp));
    const size_t ab = q->precision == QS_C64 ? sizeof(float2) : sizeof(double2);
    const size_t lds = ((size_t)1 << p.tile_d) * ab;
    const unsigned block = 1u << (p.tile_d - kRegBits);
    // as many blocks as stay resident, so each walks many tiles
    static std::map<std::tuple<int, int, int>, int> resident;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(q->device, q->precision, p.tile_d);
    auto it = resident.find(key);
    if (it == resident.end()) {
        int per_cu = 0, cus = 0;
        const hipError_t e1 =
            q->precision == QS_C64
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_step<float>, (int)block, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_step<double>, (int)block, lds);
        const hipError_t e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, q->device);
        if (e1 != hipSuccess || e2 != hipSuccess || per_cu < 1 || cus < 1)
            return fail(QS_E_HIP, "occupancy query for the tile kernel failed");
        it = resident.emplace(key, per_cu * cus).first;
    }
    const unsigned grid = grid_for(ta.num_tiles, 1, (uint64_t)it->second);
    if (q->precision == QS_C64)
        hipLaunchKernelGGL(k_tile_step<float>, dim3(grid), dim3(block), lds, q->stream, (float2 *)q->amps, ta, ph, ops,
                           (const float2 *)mats);
    else
        hipLaunchKernelGGL(k_tile_step<double>, dim3(grid), dim3(block), lds, q->stream, (double2 *)q->amps, ta, ph,
                           ops, (const double2 *)mats);
    QS_LAUNCH_CHECK();
    return QS_OK;
}

}  // namespace qs
