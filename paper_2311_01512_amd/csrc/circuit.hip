// Recorded circuits: the plain per-gate pass list, or gates fused into dense
// k-qubit blocks (FP64 products on the host), with every pass's matrix kept
// on the device in the layout of the kernel that runs it.
#include "circuit.hpp"

#include <algorithm>
#include <cmath>

namespace qs {

// Dense matrix of a gadget exp(i theta P) on its non-identity targets, in
// the order of those targets: cos(theta) 1 + i sin(theta) P, with
// P[r][c] = prod_q sigma_q[r_q][c_q] (Sec. "Pauli gadget").
static std::vector<cd> gadget_matrix(const std::vector<int> &codes, double theta)
{
    static const cd sig[4][2][2] = {{{1, 0}, {0, 1}},
                                    {{0, 1}, {1, 0}},
                                    {{0, cd(0, -1)}, {cd(0, 1), 0}},
                                    {{1, 0}, {0, -1}}};
    const int n = (int)codes.size(), D = 1 << n;
    std::vector<cd> G((size_t)D * D);
    const double c = std::cos(theta), s = std::sin(theta);
    for (int r = 0; r < D; r++)
        for (int col = 0; col < D; col++) {
            cd p = 1.0;
            for (int q = 0; q < n; q++) p *= sig[codes[q]][(r >> q) & 1][(col >> q) & 1];
            G[(size_t)r * D + col] = cd(0, s) * p + (r == col ? cd(c, 0) : cd(0, 0));
        }
    return G;
}

// The op written densely on the block qubits B (ascending; bit p <-> B[p]),
// controls expanded: identity on columns whose control bits are not all 1.
static std::vector<cd> embed_in_block(const CircOp &op, const std::vector<int> &B)
{
    std::vector<int> targs = op.targs, ctrls = op.ctrls;
    std::vector<cd> M = op.M;
    if (op.gadget) {
        std::vector<int> codes;
        targs.clear();
        for (size_t k = 0; k < op.targs.size(); k++)
            if (op.paulis[k] != 0) {
                targs.push_back(op.targs[k]);
                codes.push_back(op.paulis[k]);
            }
        M = gadget_matrix(codes, op.theta);
        ctrls.clear();
    }
    auto pos = [&](int qb) { return (int)(std::find(B.begin(), B.end(), qb) - B.begin()); };
    const int n = (int)B.size(), D = 1 << n, nt = (int)targs.size(), d = 1 << nt;
    int cmask = 0, tmask = 0;
    for (int c : ctrls) cmask |= 1 << pos(c);
    std::vector<int> tp(nt);
    for (int q = 0; q < nt; q++) {
        tp[q] = pos(targs[q]);
        tmask |= 1 << tp[q];
    }
    std::vector<cd> E((size_t)D * D, cd(0, 0));
    for (int col = 0; col < D; col++) {
        if ((col & cmask) != cmask) {
            E[(size_t)col * D + col] = 1.0;
            continue;
        }
        int l = 0;
        for (int q = 0; q < nt; q++) l |= ((col >> tp[q]) & 1) << q;
        for (int j = 0; j < d; j++) {
            int row = col & ~tmask;
            for (int q = 0; q < nt; q++) row |= ((j >> q) & 1) << tp[q];
            E[(size_t)row * D + col] += M[(size_t)j * d + l];
        }
    }
    return E;
}

static std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, int D)
{
    std::vector<cd> C((size_t)D * D, cd(0, 0));
    for (int i = 0; i < D; i++)
        for (int k = 0; k < D; k++) {
            const cd a = A[(size_t)i * D + k];
            if (a == cd(0, 0)) continue;
            for (int j = 0; j < D; j++) C[(size_t)i * D + j] += a * B[(size_t)k * D + j];
        }
    return C;
}

}  // namespace qs

using namespace qs;


namespace qs {

Pass single_pass(const CircOp &op)
{
    Pass p{};
    p.members = 1;
    if (op.gadget) {
        p.gadget = true;
        p.gtargs = op.targs;
        p.paulis = op.paulis;
        p.theta = op.theta;
    } else {
        p.gadget = false;
        p.ctrls = op.ctrls;
        p.Ms = permute_to_sorted(op.M, op.targs, p.sorted_targs);
    }
    return p;
}

// Greedy fusion: start a block at the earliest unplaced fusable op and pull
// in later ops while the qubit set stays within k and the op commutes with
// every skipped op (no shared qubit).
static void fuse(qs_circuit *c, int k)
{
    const int n_ops = (int)c->ops.size();
    std::vector<char> placed(n_ops, 0);
    std::vector<std::vector<int>> sup(n_ops);
    for (int i = 0; i < n_ops; i++) sup[i] = c->ops[i].support();
    const int lookahead = 256;
    for (int i = 0; i < n_ops; i++) {
        if (placed[i]) continue;
        placed[i] = 1;
        if ((int)sup[i].size() > k || sup[i].empty()) {
            c->passes.push_back(single_pass(c->ops[i]));
            continue;
        }
        std::vector<int> B = sup[i];
        std::vector<int> members{i};
        uint64_t blocked = 0;
        for (int j = i + 1; j < n_ops && j < i + lookahead; j++) {
            if (placed[j]) continue;
            uint64_t sj = 0;
            for (int qb : sup[j]) sj |= 1ULL << qb;
            if (sj & blocked) {
                blocked |= sj;
            } else {
                std::vector<int> U = B;
                for (int qb : sup[j])
                    if (std::find(U.begin(), U.end(), qb) == U.end()) U.push_back(qb);
                if ((int)U.size() <= k && !sup[j].empty()) {
                    B = U;
                    members.push_back(j);
                    placed[j] = 1;
                } else {
                    blocked |= sj;
                }
            }
            if (__builtin_popcountll(blocked) >= c->index_bits) break;
        }
        if (members.size() == 1) {
            c->passes.push_back(single_pass(c->ops[i]));
            continue;
        }
        std::sort(B.begin(), B.end());
        const int D = 1 << B.size();
        std::vector<cd> G((size_t)D * D, cd(0, 0));
        for (int d = 0; d < D; d++) G[(size_t)d * D + d] = 1.0;
        for (int m : members) G = matmul(embed_in_block(c->ops[m], B), G, D);
        Pass p{};
        p.gadget = false;
        p.sorted_targs = B;
        p.Ms = G;
        p.members = (int)members.size();
        c->passes.push_back(p);
    }
}

}  // namespace qs

extern "C" {

int qs_circuit_create(int num_qubits, qs_circuit **out)
{
    if (!out) return fail(QS_E_ARG, "null output pointer");
    if (num_qubits < 1 || num_qubits > 40) return fail(QS_E_ARG, "qubit count out of range");
    *out = new (std::nothrow) qs_circuit{};
    if (!*out) return fail(QS_E_ALLOC, "host allocation failed");
    (*out)->num_qubits = num_qubits;
    (*out)->index_bits = num_qubits;
    return QS_OK;
}

int qs_circuit_create_density(int num_qubits, qs_circuit **out)
{
    if (!out) return fail(QS_E_ARG, "null output pointer");
    if (num_qubits < 1 || num_qubits > 20) return fail(QS_E_ARG, "qubit count out of range");
    *out = new (std::nothrow) qs_circuit{};
    if (!*out) return fail(QS_E_ALLOC, "host allocation failed");
    (*out)->num_qubits = num_qubits;
    (*out)->is_density = 1;
    (*out)->index_bits = 2 * num_qubits;
    return QS_OK;
}

int qs_circuit_destroy(qs_circuit *c)
{
    if (!c) return QS_OK;
    release_specialized(c);   // waits for queued passes first
    if (c->dev) (void)hipFree(c->dev);
    for (auto &u : c->uses) (void)hipEventDestroy((hipEvent_t)u.second);
    delete c;
    return QS_OK;
}

int qs_circuit_add_unitary(qs_circuit *c, const int *ctrls, int num_ctrls, const int *targs, int num_targs,
                           const double *matrix)
{
    if (!c || !matrix || !targs || (num_ctrls > 0 && !ctrls)) return fail(QS_E_ARG, "null argument");
    if (num_targs < 1 || num_targs > 6 || num_ctrls < 0) return fail(QS_E_ARG, "1 to 6 targets supported per gate");
    std::vector<int> all(ctrls, ctrls + num_ctrls);
    all.insert(all.end(), targs, targs + num_targs);
    std::string why;
    if (!valid_qubits(all.data(), (int)all.size(), c->num_qubits, why)) return fail(QS_E_ARG, why);
    if ((int)all.size() > kMaxInsert) return fail(QS_E_ARG, "too many controls");
    CircOp op{};
    op.gadget = false;
    op.ctrls.assign(ctrls, ctrls + num_ctrls);
    op.targs.assign(targs, targs + num_targs);
    const size_t D = (size_t)1 << num_targs;
    op.M.resize(D * D);
    for (size_t i = 0; i < D * D; i++) op.M[i] = cd(matrix[2 * i], matrix[2 * i + 1]);
    if (c->is_density) {
        // U on (c, t) of the Choi vector, then conj(U) on (c + N, t + N)
        // (Sec. "density matrices", unitaries on the Choi vector)
        CircOp hi = op;
        for (int &x : hi.ctrls) x += c->num_qubits;
        for (int &x : hi.targs) x += c->num_qubits;
        for (auto &x : hi.M) x = std::conj(x);
        c->ops.push_back(std::move(op));
        c->ops.push_back(std::move(hi));
    } else {
        c->ops.push_back(std::move(op));
    }
    c->compiled = false;
    return QS_OK;
}

int qs_circuit_add_pauli_gadget(qs_circuit *c, const int *targs, const int *paulis, int num_targs, double theta)
{
    if (!c || !targs || !paulis || num_targs < 1) return fail(QS_E_ARG, "need at least one target");
    std::string why;
    if (!valid_qubits(targs, num_targs, c->num_qubits, why)) return fail(QS_E_ARG, why);
    for (int k = 0; k < num_targs; k++)
        if (paulis[k] < 0 || paulis[k] > 3) return fail(QS_E_ARG, "Pauli codes are 0..3");
    CircOp op{};
    op.gadget = true;
    op.targs.assign(targs, targs + num_targs);
    op.paulis.assign(paulis, paulis + num_targs);
    op.theta = theta;
    if (c->is_density) {
        // conj(exp(i theta P)) = exp(i (-1)^(m+1) theta P), m = #Y, on t + N
        CircOp hi = op;
        hi.theta = -theta;
        for (int x : hi.paulis)
            if (x == 2) hi.theta = -hi.theta;
        for (int &x : hi.targs) x += c->num_qubits;
        c->ops.push_back(std::move(op));
        c->ops.push_back(std::move(hi));
    } else {
        c->ops.push_back(std::move(op));
    }
    c->compiled = false;
    return QS_OK;
}

// A superoperator S (4^n x 4^n) on the Choi vector's qubits (t, t + N).
static int add_superop_matrix(qs_circuit *c, const int *targs, int num_targs, std::vector<cd> S)
{
    CircOp op{};
    op.gadget = false;
    op.targs.assign(targs, targs + num_targs);
    for (int i = 0; i < num_targs; i++) op.targs.push_back(targs[i] + c->num_qubits);
    op.M = std::move(S);
    c->ops.push_back(std::move(op));
    c->compiled = false;
    return QS_OK;
}

int qs_circuit_add_superop(qs_circuit *c, const int *targs, int num_targs, const double *superop)
{
    if (!c || !targs || !superop) return fail(QS_E_ARG, "null argument");
    if (!c->is_density) return fail(QS_E_PRECOND, "superoperators belong to density circuits");
    if (num_targs < 1 || num_targs > 3) return fail(QS_E_ARG, "1 to 3 targets supported");
    std::string why;
    if (!valid_qubits(targs, num_targs, c->num_qubits, why)) return fail(QS_E_ARG, why);
    const size_t D = (size_t)1 << (2 * num_targs);
    std::vector<cd> S(D * D);
    for (size_t i = 0; i < D * D; i++) S[i] = cd(superop[2 * i], superop[2 * i + 1]);
    return add_superop_matrix(c, targs, num_targs, std::move(S));
}

int qs_circuit_add_kraus_map(qs_circuit *c, const int *targs, int num_targs, const double *kraus, int num_ops)
{
    if (!c || !targs || !kraus) return fail(QS_E_ARG, "null argument");
    if (!c->is_density) return fail(QS_E_PRECOND, "Kraus maps belong to density circuits");
    if (num_targs < 1 || num_targs > 3) return fail(QS_E_ARG, "1 to 3 targets supported");
    if (num_ops < 1) return fail(QS_E_ARG, "need at least one Kraus operator");
    std::string why;
    if (!valid_qubits(targs, num_targs, c->num_qubits, why)) return fail(QS_E_ARG, why);
    const size_t d = (size_t)1 << num_targs;
    std::vector<std::vector<cd>> ks(num_ops, std::vector<cd>(d * d));
    for (int m = 0; m < num_ops; m++)
        for (size_t i = 0; i < d * d; i++) ks[m][i] = cd(kraus[2 * (m * d * d + i)], kraus[2 * (m * d * d + i) + 1]);
    return add_superop_matrix(c, targs, num_targs, superop_of_kraus(ks, num_targs));
}

int qs_circuit_compile(qs_circuit *c, int fuse_k, int precision)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (precision != QS_C64 && precision != QS_C128) return fail(QS_E_ARG, "bad precision");
    const bool tiles = fuse_k >= 8 && fuse_k <= kTileDimMax;
    if (fuse_k != 0 && !tiles && (fuse_k < 2 || fuse_k > 6))
        return fail(QS_E_ARG, "fuse_k is 0, 2..6 (dense blocks) or 8.." + std::to_string(kTileDimMax) + " (tiles)");
    if (tiles && fuse_k > tile_dim_limit(precision))
        return fail(QS_E_ARG, "tile of 2^" + std::to_string(fuse_k) + " amplitudes exceeds the LDS of a block");
    release_specialized(c);
    c->passes.clear();
    if (fuse_k == 0) {
        for (const auto &op : c->ops) c->passes.push_back(single_pass(op));
    } else if (tiles) {
        plan_tiles(c, fuse_k, precision);
    } else {
        fuse(c, fuse_k);
    }
    // device copies of every pass's tables, in its kernel's layout
    size_t total = 0;
    for (auto &p : c->passes) {
        if (p.gadget) continue;
        if (p.tile) {
            p.has_dev = true;
            p.dev_offset = total;
            total += (tile_pass_bytes(p, precision) + 255) & ~size_t(255);
            continue;
        }
        const int nt = (int)p.sorted_targs.size();
        p.kernel = choose_dense_kernel(precision, nt);
        const size_t b = dense_matrix_bytes(precision, nt, p.kernel);
        p.has_dev = b > 0;
        p.dev_offset = total;
        total += (b + 255) & ~size_t(255);
    }
    if (c->dev) {
        wait_circuit_uses(c);
        (void)hipFree(c->dev);
        c->dev = nullptr;
    }
    if (total > 0) {
        std::vector<unsigned char> host(total, 0);
        for (auto &p : c->passes) {
            if (p.tile)
                pack_tile_pass(p, precision, host.data() + p.dev_offset);
            else if (!p.gadget && p.has_dev)
                pack_dense(precision, (int)p.sorted_targs.size(), p.kernel, p.Ms, host.data() + p.dev_offset);
        }
        if (hipMalloc(&c->dev, total) != hipSuccess) {
            (void)hipGetLastError();
            c->dev = nullptr;
            return fail(QS_E_ALLOC, "device allocation of circuit matrices failed");
        }
        QS_HIP(hipMemcpy(c->dev, host.data(), total, hipMemcpyHostToDevice));
        QS_HIP(hipGetDevice(&c->device));
    }
    c->dev_bytes = total;
    c->precision = precision;
    c->fuse_k = fuse_k;
    c->compiled = true;
    return QS_OK;
}

int qs_circuit_stats(const qs_circuit *c, int *num_ops, int *num_passes, uint64_t *logical_updates,
                     int *blocks_by_width)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (num_ops) *num_ops = (int)c->ops.size();
    if (num_passes) *num_passes = c->compiled ? (int)c->passes.size() : -1;
    if (logical_updates) {
        uint64_t u = 0;
        for (const auto &op : c->ops)
            u += op.gadget ? (1ULL << c->index_bits) : (1ULL << (c->index_bits - (int)op.ctrls.size()));
        *logical_updates = u;
    }
    if (blocks_by_width) {
        for (int i = 0; i < 7; i++) blocks_by_width[i] = 0;
        for (const auto &p : c->passes)
            if (!p.tile) blocks_by_width[p.gadget ? 0 : (int)p.sorted_targs.size()]++;
    }
    return QS_OK;
}

int qs_apply_circuit(qs_qureg *q, qs_circuit *c)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    return qs_apply_circuit_passes(q, c, 0, (int)c->passes.size());
}

}  // extern "C"

namespace qs {

// FNV-1a over the recorded ops (structure and matrix bits): the key under
// which the autotuner caches its choice for a circuit.
uint64_t circuit_fingerprint(const qs_circuit *c)
{
    uint64_t h = 1469598103934665603ULL;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; i++) {
            h ^= b[i];
            h *= 1099511628211ULL;
        }
    };
    mix(&c->num_qubits, sizeof(int));
    mix(&c->is_density, sizeof(int));
    for (const auto &op : c->ops) {
        mix(&op.gadget, sizeof(bool));
        for (int x : op.ctrls) mix(&x, sizeof(int));
        for (int x : op.targs) mix(&x, sizeof(int));
        for (int x : op.paulis) mix(&x, sizeof(int));
        mix(&op.theta, sizeof(double));
        if (!op.M.empty()) mix(op.M.data(), op.M.size() * sizeof(cd));
    }
    return h;
}

int circuit_num_qubits(const qs_circuit *c) { return c->num_qubits; }

int note_circuit_use(qs_circuit *c, hipStream_t s)
{
    hipEvent_t ev = nullptr;
    for (auto &u : c->uses)
        if (u.first == (void *)s) ev = (hipEvent_t)u.second;
    if (!ev) {
        QS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->uses.emplace_back((void *)s, (void *)ev);
    }
    QS_HIP(hipEventRecord(ev, s));
    return QS_OK;
}

void wait_circuit_uses(qs_circuit *c)
{
    for (auto &u : c->uses) (void)hipEventSynchronize((hipEvent_t)u.second);
}

}  // namespace qs

extern "C" {

int qs_circuit_pass_info(const qs_circuit *c, int index, int *kernel, int *num_targs, int *num_ctrls, int *members,
                         int *phases)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (!c->compiled) return fail(QS_E_PRECOND, "circuit is not compiled");
    if (index < 0 || index >= (int)c->passes.size()) return fail(QS_E_ARG, "pass index out of range");
    const Pass &p = c->passes[index];
    int k, nt, nc;
    if (p.tile) {
        k = 4;
        nt = p.tile_d;
        nc = 0;
    } else if (p.gadget) {
        bool xy = false;
        nt = 0;
        for (int code : p.paulis) {
            if (code == 1 || code == 2) xy = true;
            if (code != 0) nt++;
        }
        k = xy ? 0 : 1;
        nc = 0;
    } else {
        nt = (int)p.sorted_targs.size();
        nc = (int)p.ctrls.size();
        const uint64_t groups = 1ULL << (c->index_bits - nt - nc);
        const bool mfma = p.kernel == kDenseMfma && c->precision == QS_C64 && nt >= 4 && groups >= 16;
        k = mfma ? 3 : 2;
    }
    if (kernel) *kernel = k;
    if (num_targs) *num_targs = nt;
    if (num_ctrls) *num_ctrls = nc;
    if (members) *members = p.members;
    if (phases) *phases = p.tile ? (int)p.phases.size() : 1;
    return QS_OK;
}

int qs_apply_circuit_passes(qs_qureg *q, qs_circuit *c, int first, int count)
{
    if (!q || !c) return fail(QS_E_ARG, "null argument");
    if (q->is_density != c->is_density)
        return fail(QS_E_PRECOND, c->is_density ? "density circuits apply to density matrices"
                                                : "statevector circuits apply to statevectors");
    if (q->num_qubits != c->num_qubits) return fail(QS_E_ARG, "qubit counts differ");
    if (!c->compiled) return fail(QS_E_PRECOND, "circuit is not compiled");
    if (c->precision != q->precision) return fail(QS_E_TYPE, "circuit compiled for the other precision");
    if (c->dev && c->device != q->device) return fail(QS_E_PRECOND, "circuit matrices live on another device");
    if (first < 0 || count < 0 || first + count > (int)c->passes.size()) return fail(QS_E_ARG, "pass range out of bounds");
    for (int pi = first; pi < first + count; pi++) {
        const Pass &p = c->passes[pi];
        int rc;
        if (p.tile) {
            rc = launch_tile_pass(q, p, (const unsigned char *)c->dev + p.dev_offset);
        } else if (p.gadget) {
            rc = apply_raw_gadget(q, p.gtargs, p.paulis, p.theta);
        } else {
            const void *dev = p.has_dev ? (const void *)((const unsigned char *)c->dev + p.dev_offset) : nullptr;
            rc = launch_dense(q, p.ctrls, p.sorted_targs, p.Ms, dev, p.kernel);
        }
        if (rc != QS_OK) return rc;
    }
    return count > 0 ? note_circuit_use(c, q->stream) : QS_OK;
}

}  // extern "C"
