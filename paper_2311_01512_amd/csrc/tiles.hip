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
#include "tile_dev.hpp"

#include <algorithm>
#include <cstdlib>
#include <deque>
#include <map>
#include <string>
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
// Member fusion: an uncontrolled dense gate whose targets lie inside those
// of another uncontrolled dense gate of the step joins it as one operator,
// the FP64 product of the two, when every member between them commutes with
// the one that moves (so the product applies at the other's place).  Fewer
// operators, the same map: a one-qubit gate next to a two-qubit gate on that
// qubit, or a density matrix's U and conj(U) next to a channel on (t, t + N),
// cost one matrix instead of two or three.  QS_TILE_FUSE=0 turns it off.
static bool tile_fuse_enabled()
{
    static const bool on = [] {
        const char *e = std::getenv("QS_TILE_FUSE");
        return !(e && std::string(e) == "0");
    }();
    return on;
}

// A's matrix on the target list `tt` (a superset of A's targets): identity
// on the others.  Matrices are row-major, bit q of an index <-> target q.
static std::vector<cd> embed_matrix(const CircOp &a, const std::vector<int> &tt)
{
    const size_t D = (size_t)1 << tt.size(), Da = (size_t)1 << a.targs.size();
    std::vector<int> pos(a.targs.size());
    uint32_t amask = 0;
    for (size_t q = 0; q < a.targs.size(); q++) {
        pos[q] = (int)(std::find(tt.begin(), tt.end(), a.targs[q]) - tt.begin());
        amask |= 1u << pos[q];
    }
    auto sub = [&](size_t r) {
        size_t v = 0;
        for (size_t q = 0; q < pos.size(); q++) v |= ((r >> pos[q]) & 1u) << q;
        return v;
    };
    std::vector<cd> m(D * D, cd(0, 0));
    for (size_t r = 0; r < D; r++)
        for (size_t c = 0; c < D; c++)
            if ((r & ~(size_t)amask) == (c & ~(size_t)amask)) m[r * D + c] = a.M[sub(r) * Da + sub(c)];
    return m;
}

static std::vector<const CircOp *> fuse_members(const std::vector<const CircOp *> &in, std::deque<CircOp> &store)
{
    std::vector<const CircOp *> L = in;
    if (!tile_fuse_enabled()) return L;
    auto dense = [](const CircOp *o) { return !o->gadget && o->ctrls.empty(); };
    auto inside = [](const CircOp *a, const CircOp *b) {   // targets of a within those of b
        for (int t : a->targs)
            if (std::find(b->targs.begin(), b->targs.end(), t) == b->targs.end()) return false;
        return true;
    };
    std::vector<char> alive(L.size(), 1);
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t j = 0; j < L.size(); j++) {
            if (!alive[j] || !dense(L[j])) continue;
            const CircOp *X = L[j];
            const OpMasks mx = op_masks(*X);
            for (size_t i = j; i-- > 0;) {
                if (!alive[i]) continue;
                const CircOp *Y = L[i];
                if (dense(Y) && (inside(Y, X) || inside(X, Y))) {
                    const bool fwd = inside(Y, X);   // Y moves forward to X, else X back to Y
                    const OpMasks mm = op_masks(fwd ? *Y : *X);
                    bool ok = true;
                    for (size_t k = i + 1; k < j && ok; k++)
                        if (alive[k] && !ops_commute(mm, op_masks(*L[k]))) ok = false;
                    if (ok) {
                        CircOp f;
                        f.gadget = false;
                        f.theta = 0.0;
                        f.targs = fwd ? X->targs : Y->targs;
                        const size_t D = (size_t)1 << f.targs.size();
                        const std::vector<cd> a = embed_matrix(*Y, f.targs), b = embed_matrix(*X, f.targs);
                        f.M.assign(D * D, cd(0, 0));
                        for (size_t r = 0; r < D; r++)   // X after Y: b a
                            for (size_t k = 0; k < D; k++) {
                                const cd brk = b[r * D + k];
                                if (brk == cd(0, 0)) continue;
                                for (size_t c = 0; c < D; c++) f.M[r * D + c] += brk * a[k * D + c];
                            }
                        store.push_back(std::move(f));
                        if (fwd) {
                            L[j] = &store.back();
                            alive[i] = 0;
                        } else {
                            L[i] = &store.back();
                            alive[j] = 0;
                        }
                        changed = true;
                    }
                    break;
                }
                if (!ops_commute(op_masks(*Y), mx)) break;
            }
        }
    }
    std::vector<const CircOp *> out;
    for (size_t k = 0; k < L.size(); k++)
        if (alive[k]) out.push_back(L[k]);
    return out;
}

static void encode_step(Pass &p, const Echelon &E, const std::vector<const CircOp *> &recorded, bool mfma)
{
    std::deque<CircOp> fused;
    const std::vector<const CircOp *> members = fuse_members(recorded, fused);
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
    // A phase takes, in order, every remaining member that fits it and
    // commutes with each remaining member it jumps over.
    std::vector<size_t> remaining(members.size());
    for (size_t m = 0; m < members.size(); m++) remaining[m] = m;
    std::vector<OpMasks> mmask(members.size());
    for (size_t m = 0; m < members.size(); m++) mmask[m] = op_masks(*members[m]);
    while (!remaining.empty()) {
        PhaseBuild B;
        std::vector<size_t> chosen, rest;
        std::vector<int> mode;
        for (size_t m : remaining) {
            bool free = true;
            for (size_t k : rest)
                if (!ops_commute(mmask[m], mmask[k])) {
                    free = false;
                    break;
                }
            int md = -1;
            if (free) md = try_fit(B, m);
            if (md >= 0) {
                chosen.push_back(m);
                mode.push_back(md);
            } else {
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
    p.members = (int)recorded.size();
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
    std::vector<OpMasks> masks(n_ops);
    std::vector<std::vector<uint64_t>> needs(n_ops);
    for (int i = 0; i < n_ops; i++) {
        masks[i] = op_masks(c->ops[i]);
        needs[i] = needed_vectors(c->ops[i]);
    }
    // Admission rules for one step.  Rule g < 0: one greedy sweep over the
    // window.  Rule g >= 0: a first sweep admits only operators that grow the
    // span by at most g dimensions (the step's first operator always), then
    // the greedy sweep.  Either way an operator joins a step only if it
    // commutes with every earlier operator left out, so it also commutes
    // with every member placed after it in circuit order: the member list
    // is a valid order of application.
    auto build_step = [&](int i, int g, std::vector<char> &placed, Echelon &E,
                          std::vector<const CircOp *> &members) {
        for (int b = 0; b < C; b++) E.add(1ULL << b);
        for (int sweep = g < 0 ? 1 : 0; sweep < 2; sweep++) {
            // operators the step leaves out: a later operator joins only if
            // it commutes with every one of them
            std::vector<int> skipped;
            for (int j = i; j < n_ops && j < i + lookahead; j++) {
                if (placed[j]) continue;
                const CircOp &op = c->ops[j];
                bool free = true;
                for (int k : skipped)
                    if (!ops_commute(masks[j], masks[k])) {
                        free = false;
                        break;
                    }
                if (!free) {
                    skipped.push_back(j);
                    continue;
                }
                const int dim = E.dim_with(needs[j]);
                const bool fits = absorbable(op, mfma) && op.ctrls.size() <= 4 && dim <= T &&
                                  (sweep == 1 || j == i || dim - E.dim() <= g);
                if (fits) {
                    for (uint64_t x : needs[j]) E.add(x);
                    members.push_back(&op);
                    placed[j] = 1;
                } else {
                    skipped.push_back(j);
                }
            }
        }
    };
    // one plan per rule, the same rule for every step
    auto plan = [&](int rule, std::vector<Pass> &out) {
        std::vector<char> placed(n_ops, 0);
        for (int i = 0; i < n_ops; i++) {
            if (placed[i]) continue;
            const CircOp &first = c->ops[i];
            // registers need a tile of more than kRegBits dimensions; controls
            // beyond the 4 a tile operator carries, or gates of more than 3
            // targets, run as passes of their own
            if (T <= kRegBits || !absorbable(first, mfma) || first.ctrls.size() > 4) {
                placed[i] = 1;
                out.push_back(single_pass(first));
                continue;
            }
            Echelon E;
            std::vector<const CircOp *> members;
            build_step(i, rule, placed, E, members);
            // fill the tile to T dimensions with the lowest free qubits: longer
            // contiguous runs, fewer and larger tiles
            for (int b = C; b < N && E.dim() < T; b++) E.add(1ULL << b);
            Pass p{};
            encode_step(p, E, members, mfma);
            out.push_back(std::move(p));
        }
    };
    // the plan with the fewest passes wins (ties to the plain greedy)
    std::vector<Pass> best;
    plan(-1, best);
    for (int rule : {0, 1}) {
        std::vector<Pass> alt;
        plan(rule, alt);
        if (alt.size() < best.size()) best.swap(alt);
    }
    for (Pass &p : best) c->passes.push_back(std::move(p));
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t tile_mats_offset(const Pass &p)
{
    return align256(p.phases.size() * sizeof(RPhase)) + align256(p.rops.size() * sizeof(ROp));
}

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
    int chunk;           // each block walks a run of consecutive tiles (else a stride)
};

// The generic tile-step kernel: phases and operators read from the pass's
// device tables, one switch per operator (see tile_walk).
template <typename R>
__global__ __launch_bounds__(1024) void k_tile_step(C2<R> *__restrict__ a, TileArgs ta, const RPhase *__restrict__ ph,
                                                     const ROp *__restrict__ ops, const C2<R> *__restrict__ mats)
{
    extern __shared__ unsigned char lds_raw[];
    const int lb = ta.d - kRegBits;
    const RPhase &first = ph[0];
    tile_walk<R>(a, ta.num_tiles, ta.plan, first, ph[ta.nph - 1], lb, ta.chunk != 0, [&](C2<R>(&x)[kRegs], uint64_t base) {
        uint32_t tau = tau_of(threadIdx.x, first);
        for (int p = 0; p < ta.nph; p++) {
            const RPhase &P = ph[p];
            if (p > 0) tau = tile_exchange<R>(x, lds_raw, tau, ph[p - 1], P);
            const int end = P.first_op + P.num_ops;
            for (int o = P.first_op; o < end; o++) apply_reg_op<R>(x, ops[o], tau, base, mats);
        }
    });
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
    // grid: resident blocks each walking a run of consecutive tiles, resident
    // blocks walking by a fixed stride, or one block per tile
    const int policy = tile_grid_policy(p.tile_d);
    ta.chunk = policy == kTileGridChunk ? 1 : 0;
    if (p.jit_fn) {
        // the step's own kernel: phases and operators compiled in
        void *a = q->amps;
        uint64_t nt = ta.num_tiles;
        const void *mp = mats;
        int chunk = ta.chunk;
        void *args[] = {&a, &nt, &mp, &chunk};
        const uint64_t ck = policy == kTileGridChunk ? tile_chunk() : 0;
        const unsigned grid = policy == kTileGridPerTile ? grid_for(nt << (p.tile_d - kRegBits), block)
                              : ck ? grid_for(((nt + ck - 1) / ck) * block, block)
                                   : grid_for(nt, 1, p.jit_grid);
        QS_HIP(hipModuleLaunchKernel((hipFunction_t)p.jit_fn, grid, 1, 1, block, 1, 1, p.jit_lds, q->stream, args,
                                     nullptr));
        return QS_OK;
    }
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
    const uint64_t ck = policy == kTileGridChunk ? tile_chunk() : 0;
    const unsigned grid = policy == kTileGridPerTile ? grid_for(ta.num_tiles << (p.tile_d - kRegBits), block)
                          : ck ? grid_for(((ta.num_tiles + ck - 1) / ck) * block, block)
                               : grid_for(ta.num_tiles, 1, (uint64_t)it->second);
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
