// Run-time specialisation of tile steps.  The generic tile-step kernel reads
// each step's phases and operators from device tables and dispatches every
// operator through a switch; here each step of a compiled circuit becomes a
// kernel of its own, generated as HIP source in which the phases and
// operators are compile-time constants (the same device functions as the
// generic kernel, tile_dev.hpp), compiled for the device (rtc.hip) and
// loaded as modules.  Operator dispatch, operator-field loads and the
// register copies at the merge of the switch's arms disappear; the results
// are those of the generic kernel.
#include "circuit.hpp"

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>


namespace qs {

namespace {

std::string hexd(double v)
{
    char b[64];
    std::snprintf(b, sizeof b, "%a", v);
    return b;
}

std::string hexf(float v)
{
    char b[64];
    std::snprintf(b, sizeof b, "%af", (double)v);
    return b;
}

std::string u64(uint64_t v)
{
    char b[32];
    std::snprintf(b, sizeof b, "0x%" PRIx64 "ull", v);
    return b;
}

std::string u32(uint32_t v)
{
    char b[32];
    std::snprintf(b, sizeof b, "0x%xu", v);
    return b;
}

template <typename T, typename F>
std::string list(const T *v, int n, F f)
{
    std::string s = "{";
    for (int i = 0; i < n; i++) s += (i ? ", " : "") + f(v[i]);
    return s + "}";
}

std::string phase_init(const RPhase &p)
{
    auto i32 = [](int v) { return std::to_string(v); };
    std::ostringstream o;
    o << "{" << list(p.rho, kRegs, u32) << ", " << list(p.lo, kRegBits + 2, u32) << ", " << p.nlo << ", " << p.c4
      << ", " << p.c5 << ", " << u32(p.pad_) << ", " << list(p.yaddr, kRegs, u64) << ", "
      << list(p.taddr, kTileDimMax, u64) << ", " << i32(p.first_op) << ", " << i32(p.num_ops) << "}";
    return o.str();
}

std::string op_init(const ROp &r)
{
    auto i32 = [](int v) { return std::to_string(v); };
    std::ostringstream o;
    o << "{" << r.code << ", " << r.nc << ", " << list(r.cq, 4, i32) << ", " << list(r.cm, 4, u32) << ", "
      << u64(r.qtab) << ", " << u64(r.yz) << ", " << u32(r.yzm) << ", " << u32(r.gy) << ", " << r.mat << ", "
      << u32(r.hsel) << ", " << hexd(r.cs) << ", " << hexd(r.cre) << ", " << hexd(r.cim) << ", " << hexd(r.pre)
      << ", " << hexd(r.pim) << ", " << hexf(r.fcs) << ", " << hexf(r.fcre) << ", " << hexf(r.fcim) << ", "
      << hexf(r.fpre) << ", " << hexf(r.fpim) << "}";
    return o.str();
}

// Register bits of a dense (codes 1-7, 17-23) or sparse (64+) register
// operator, 0 for other codes.
int matrix_bits(int c)
{
    if (c >= 1 && c <= 7) return c;
    if (c >= 17 && c <= 23) return c - 16;
    if (c >= 64) return (c - 64) >> 2;
    return 0;
}

// The matrix of a dense or sparse register operator as a constexpr array
// `M` holding the values of the pass's device table (FP32 for complex64).
std::string matrix_init(const Pass &p, const ROp &r, bool f32)
{
    const int bits = matrix_bits(r.code);
    const int n = 1 << (2 * __builtin_popcount((unsigned)bits));
    std::ostringstream o;
    o << "static constexpr " << (f32 ? "float2" : "double2") << " M[" << n << "] = {";
    for (int i = 0; i < n; i++) {
        const std::complex<double> &v = p.tmats[(size_t)r.mat + i];
        o << (i ? ", " : "") << (f32 ? "float2{" : "double2{");
        if (f32)
            o << hexf((float)v.real()) << ", " << hexf((float)v.imag());
        else
            o << hexd(v.real()) << ", " << hexd(v.imag());
        o << "}";
    }
    o << "};";
    return o.str();
}

// The call that applies operator `name` (a constexpr ROp) in a phase; empty
// for codes the generic kernel ignores as well.  Dense and sparse register
// operators take their matrix from the constexpr array M (the entries end up
// as instruction literals instead of loads into scalar registers).
std::string op_call(const ROp &r, const std::string &name, bool f32)
{
    const int c = r.code;
    std::ostringstream o;
    if (c >= 1 && c <= 7)
        o << "qs::reg_dense<R, " << c << ", false>(x, " << name << ", tau, base, M);";
    else if (c >= 17 && c <= 23)
        o << "qs::reg_dense<R, " << c - 16 << ", true>(x, " << name << ", tau, base, M);";
    else if (c >= 8 && c <= 15)
        o << "qs::reg_gadget<R, " << c - 8 << ">(x, " << name << ", tau, base);";
    else if (c == 16)
        o << "qs::reg_scale<R>(x, " << name << ");";
    else if (c >= 24 && c <= 31)
        o << "qs::reg_gadget_f<R, " << c - 24 << ", true>(x, " << name << ", tau, base);";
    else if (c >= 41 && c <= 47)
        o << "qs::reg_gadget_f<R, " << c - 40 << ", false>(x, " << name << ", tau, base);";
    else if (c >= 32 && c <= 38 && f32)
        o << "qs::mfma_dense<" << c - 32 << ">(x, " << name << ", tau, base, mats);";
    else if (c >= 64) {
        const int um = (c - 64) >> 2, sm = (c - 64) & 3;
        o << "qs::reg_sparse<R, " << um << ", " << sm << ">(x, M);";
    }
    return o.str();
}

// Matrix-core operators of a specialised step read their per-lane
// coefficients from LDS: the variants their register groups use are copied
// once per block, behind the tile.  (Read from global memory for every tile,
// as the generic kernel does, these loads missed L2 nearly every time.)
// Offsets and lengths in floats; `ops` maps an operator's index to its
// (mat, hsel) relative to the LDS tables.
struct MfmaStage {
    std::vector<unsigned> src, dst, len, width, lane_floats;   // width: chunk TW; lane_floats: NB * KS
    std::map<int, std::pair<int, uint32_t>> ops;
    unsigned floats = 0;
};

MfmaStage stage_mfma(const Pass &p)
{
    MfmaStage st;
    for (size_t oi = 0; oi < p.rops.size(); oi++) {
        const ROp &r = p.rops[oi];
        if (r.code < 32 || r.code > 38) continue;
        const int rm = r.code - 32;
        const int regs = 1 << __builtin_popcount((unsigned)rm);
        const unsigned lane_floats = (unsigned)(regs >= 2 ? regs / 2 : 1) * (unsigned)(2 * regs);
        const unsigned per_variant = 64u * lane_floats;
        int slot_of[4] = {-1, -1, -1, -1}, slots = 0;
        uint32_t hsel = 0;
        const unsigned first = st.floats;
        for (int u0 = 0; u0 < kRegs; u0++) {
            if (u0 & rm) continue;
            const int h = (int)((r.hsel >> (2 * u0)) & 3u);
            if (slot_of[h] < 0) {
                slot_of[h] = slots++;
                st.src.push_back(2u * (unsigned)r.mat + (unsigned)h * per_variant);
                st.dst.push_back(st.floats);
                st.len.push_back(per_variant);
                st.width.push_back(std::min(4u, lane_floats));
                st.lane_floats.push_back(lane_floats);
                st.floats += per_variant;
            }
            hsel |= (uint32_t)slot_of[h] << (2 * u0);
        }
        st.ops[(int)oi] = {(int)(first / 2), hsel};
    }
    return st;
}

// The staging of a step, empty when there is nothing to stage or the tile
// and the tables would not fit the LDS a block may have (max_lds): such a
// step reads the coefficients from global memory.
MfmaStage stage_for(const Pass &p, bool f32, size_t max_lds)
{
    if (!f32) return MfmaStage{};
    MfmaStage st = stage_mfma(p);
    if (((size_t)1 << p.tile_d) * sizeof(float2) + 4 * (size_t)st.floats > max_lds) return MfmaStage{};
    return st;
}

// Bytes of LDS a specialised step needs: the tile, then the staged tables.
size_t step_lds_bytes(const Pass &p, bool f32, size_t max_lds)
{
    return ((size_t)1 << p.tile_d) * (f32 ? sizeof(float2) : sizeof(double2)) +
           4 * (size_t)stage_for(p, f32, max_lds).floats;
}

// One kernel per tile pass, named qs_step_<index>.
std::string step_kernel(const Pass &p, int index, bool f32, size_t max_lds)
{
    const int lb = p.tile_d - kRegBits;
    const int block = 1 << lb;
    std::ostringstream o;
    const char *c2 = f32 ? "float2" : "double2";
    // the occupancy of the generic kernel (six waves per SIMD for complex64,
    // four for complex128): straight-line code would otherwise hoist loads
    // and spend registers on them
    o << "extern \"C\" __global__ __launch_bounds__(" << block << ") __attribute__((amdgpu_waves_per_eu("
      << step_waves_per_eu(f32) << "))) void qs_step_" << index << "(" << c2
      << " *__restrict__ a, unsigned long long num_tiles, const " << c2
      << " *__restrict__ mats, int chunk)\n{\n";
    o << "    using R = " << (f32 ? "float" : "double") << ";\n";
    o << "    extern __shared__ unsigned char lds_raw[];\n";
    std::vector<int> piv = p.pivots;
    for (size_t i = 1; i < piv.size(); i++)
        for (size_t j = i; j > 0 && piv[j - 1] > piv[j]; j--) std::swap(piv[j - 1], piv[j]);
    o << "    constexpr qs::InsertPlan plan = {" << piv.size() << ", {";
    for (size_t k = 0; k < piv.size(); k++) o << (k ? ", " : "") << u64((1ULL << piv[k]) - 1ULL);
    o << "}};\n";
    for (size_t k = 0; k < p.phases.size(); k++)
        o << "    constexpr qs::RPhase P" << k << " = " << phase_init(p.phases[k]) << ";\n";
    const MfmaStage st = stage_for(p, f32, max_lds);
    const size_t tile_bytes = ((size_t)1 << p.tile_d) * (f32 ? sizeof(float2) : sizeof(double2));
    if (!st.src.empty()) {
        auto ulist = [](const std::vector<unsigned> &v) {
            std::string t = "{";
            for (size_t i = 0; i < v.size(); i++) t += (i ? ", " : "") + std::to_string(v[i] / 2) + "u";
            return t + "}";
        };
        // float2 units
        o << "    const float2 *tabs = reinterpret_cast<const float2 *>(lds_raw + " << tile_bytes << ");\n";
        auto plain = [](const std::vector<unsigned> &v) {
            std::string t = "{";
            for (size_t i = 0; i < v.size(); i++) t += (i ? ", " : "") + std::to_string(v[i]) + "u";
            return t + "}";
        };
        // chunk c: float2 e of the LDS copy is floats d = 2e, 2e + 1 of lane
        // (d / W) % 64, chunk (d / W) / 64, from the lane's floats in memory
        o << "    {\n        constexpr unsigned cs[] = " << ulist(st.src) << ", cd[] = " << ulist(st.dst)
          << ", cl[] = " << ulist(st.len) << ", cw[] = " << plain(st.width) << ", cn[] = " << plain(st.lane_floats)
          << ";\n";
        o << "        float2 *dst = reinterpret_cast<float2 *>(lds_raw + " << tile_bytes << ");\n";
        o << "#pragma unroll\n        for (int c = 0; c < " << st.src.size() << "; c++)\n";
        o << "            for (unsigned e = threadIdx.x; e < cl[c]; e += " << block << "u) {\n";
        o << "                const unsigned d = 2u * e, v = d / cw[c];\n";
        o << "                dst[cd[c] + e] = mats[cs[c] + ((v & 63u) * cn[c] + (v >> 6) * cw[c] + d % cw[c]) / 2u];\n";
        o << "            }\n";
        o << "        __syncthreads();\n    }\n";
    }
    o << "    qs::tile_walk<R>(a, num_tiles, plan, P0, P" << p.phases.size() - 1 << ", " << lb
      << ", chunk != 0, [&](qs::C2<R> (&x)[qs::kRegs], uint64_t base) {\n";
    o << "        uint32_t tau = qs::tau_of(threadIdx.x, P0);\n";
    for (size_t k = 0; k < p.phases.size(); k++) {
        const RPhase &P = p.phases[k];
        if (k > 0) o << "        tau = qs::tile_exchange<R>(x, lds_raw, tau, P" << k - 1 << ", P" << k << ");\n";
        for (int oi = P.first_op; oi < P.first_op + P.num_ops; oi++) {
            ROp r = p.rops[oi];
            std::string call = op_call(r, "O", f32);
            if (call.empty()) continue;
            auto it = st.ops.find(oi);
            if (it != st.ops.end()) {
                // coefficients from the LDS tables
                r.mat = it->second.first;
                r.hsel = it->second.second;
                const int rm = r.code - 32, regs = 1 << __builtin_popcount((unsigned)rm);
                const int lane_floats = (regs >= 2 ? regs / 2 : 1) * 2 * regs;
                call = "qs::mfma_dense<" + std::to_string(rm) + ", " + std::to_string(std::min(4, lane_floats)) +
                       ">(x, O, tau, base, tabs);";
            }
            o << "        { constexpr qs::ROp O = " << op_init(r) << "; ";
            if (matrix_bits(p.rops[oi].code)) o << matrix_init(p, p.rops[oi], f32) << " ";
            o << call << " }\n";
        }
    }
    o << "    });\n}\n\n";
    return o.str();
}


}  // namespace

// Sources of the tile passes of a compiled circuit (kernel name = pass
// index), split into `chunks` files of about equal kernel counts.
std::vector<std::string> specialized_sources(const qs_circuit *c, int chunks, size_t max_lds)
{
    const bool f32 = c->precision == QS_C64;
    std::vector<int> idx;
    for (size_t i = 0; i < c->passes.size(); i++)
        if (c->passes[i].tile && !c->passes[i].phases.empty()) idx.push_back((int)i);
    chunks = std::max(1, std::min<int>(chunks, (int)idx.size()));
    std::vector<std::string> out(chunks, "#include \"tile_dev.hpp\"\n\n");
    for (size_t j = 0; j < idx.size(); j++) out[j * chunks / idx.size()] += step_kernel(c->passes[idx[j]], idx[j], f32, max_lds);
    return out;
}

void release_specialized(qs_circuit *c)
{
    if (!c->jit_modules.empty()) wait_circuit_uses(c);   // queued steps may still run these kernels
    for (auto &p : c->passes) {
        p.jit_fn = nullptr;
        p.jit_grid = 0;
        p.jit_lds = 0;
    }
    for (void *m : c->jit_modules) (void)hipModuleUnload((hipModule_t)m);
    c->jit_modules.clear();
}

int specialize_tiles(qs_circuit *c, int *num_kernels)
{
    release_specialized(c);
    int count = 0;
    for (const auto &p : c->passes)
        if (p.tile && !p.phases.empty()) count++;
    if (num_kernels) *num_kernels = count;
    if (count == 0) return QS_OK;
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    if (c->dev && c->device != dev) return fail(QS_E_PRECOND, "circuit tables live on another device");
    hipDeviceProp_t prop;
    QS_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    // several compilers at once: a few kernels per child process
    const int chunks = std::max(1, std::min(8, (count + 3) / 4));
    std::vector<std::vector<char>> codes;
    const size_t max_lds = prop.sharedMemPerBlock;
    int rc = compile_device_sources(specialized_sources(c, chunks, max_lds), arch, codes);
    if (rc != QS_OK) return rc;
    for (const auto &code : codes) {
        hipModule_t mod;
        if (hipModuleLoadData(&mod, code.data()) != hipSuccess) {
            (void)hipGetLastError();
            release_specialized(c);
            return fail(QS_E_HIP, "loading the specialised tile steps failed");
        }
        c->jit_modules.push_back(mod);
    }
    int cus = 0;
    QS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int j = 0;
    for (size_t i = 0; i < c->passes.size(); i++) {
        Pass &p = c->passes[i];
        if (!p.tile || p.phases.empty()) continue;
        // the chunk that specialized_sources put this pass in
        const hipModule_t mod = (hipModule_t)c->jit_modules[(size_t)j++ * codes.size() / count];
        hipFunction_t f = nullptr;
        const std::string name = "qs_step_" + std::to_string(i);
        if (hipModuleGetFunction(&f, mod, name.c_str()) != hipSuccess) {
            (void)hipGetLastError();
            release_specialized(c);
            return fail(QS_E_HIP, "specialised kernel " + name + " missing from its module");
        }
        int per_cu = 0;
        const int block = 1 << (p.tile_d - kRegBits);
        const size_t lds = step_lds_bytes(p, c->precision == QS_C64, max_lds);
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, block, lds) != hipSuccess || per_cu < 1) {
            release_specialized(c);
            return fail(QS_E_HIP, "occupancy query for " + name + " failed");
        }
        p.jit_fn = (void *)f;
        p.jit_grid = (unsigned)(per_cu * cus);
        p.jit_lds = (unsigned)lds;
    }
    return QS_OK;
}

}  // namespace qs

using namespace qs;

extern "C" int qs_circuit_specialize(qs_circuit *c, int *num_kernels)
{
    if (!c) return fail(QS_E_ARG, "null circuit");
    if (!c->compiled) return fail(QS_E_PRECOND, "circuit is not compiled");
    return specialize_tiles(c, num_kernels);
}
