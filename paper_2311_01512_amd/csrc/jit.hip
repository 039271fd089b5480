// Run-time specialisation of tile steps.  The generic tile-step kernel reads
// each step's phases and operators from device tables and dispatches every
// operator through a switch; here each step of a compiled circuit becomes a
// kernel of its own, generated as HIP source in which the phases and
// operators are compile-time constants (the same device functions as the
// generic kernel, tile_dev.hpp), compiled for the device by the ROCm clang
// (run as child processes, several at once) and loaded as modules.  (hiprtc
// is not used: in a process that has loaded PyTorch it resolves to the
// compiler bundled with PyTorch, whose code for these kernels spills to
// scratch memory.)  Operator dispatch, operator-field loads and the
// register copies at the merge of the switch's arms disappear; the results
// are those of the generic kernel.
#include "circuit.hpp"

#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <fstream>
#include <functional>
#include <iterator>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

// kRtcHeaderNames / kRtcHeaderSources: dev_core.hpp and tile_dev.hpp as
// strings (written by the build from the sources in this directory)
#include "qs_rtc_headers.inc"

extern char **environ;

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
      << (f32 ? 6 : 4) << "))) void qs_step_" << index << "(" << c2
      << " *__restrict__ a, unsigned long long num_tiles, const " << c2 << " *__restrict__ mats)\n{\n";
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
      << ", [&](qs::C2<R> (&x)[qs::kRegs], uint64_t base) {\n";
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

// Compiled code objects by compilation key (target, compiler, options,
// headers, source), for the process; autotuning and benchmarking compile the
// same circuit more than once.
std::mutex g_mu;
std::map<std::string, std::vector<char>> g_code;

std::string rocm_path()
{
    const char *e = std::getenv("ROCM_PATH");
    return e && *e ? e : "/opt/rocm";
}

bool write_file(const std::string &path, const std::string &text)
{
    std::ofstream f(path, std::ios::binary);
    f << text;
    return (bool)f;
}

bool read_file(const std::string &path, std::vector<char> &out)
{
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return true;
}

// 64-bit FNV-1a of `s` from offset basis `h` (names cache files only: a
// cached entry holds its whole key and is used only if that key matches).
uint64_t fnv1a(const std::string &s, uint64_t h)
{
    for (unsigned char ch : s) h = (h ^ ch) * 0x100000001b3ull;
    return h;
}

// Directory of the on-disk code-object cache: $QS_JIT_CACHE, else
// qs_jit_cache under $TMPDIR (default /tmp); empty if it cannot be made.
std::string cache_dir()
{
    const char *e = std::getenv("QS_JIT_CACHE");
    std::string d;
    if (e && *e) {
        d = e;
    } else {
        const char *t = std::getenv("TMPDIR");
        d = std::string(t && *t ? t : "/tmp") + "/qs_jit_cache";
    }
    if (mkdir(d.c_str(), 0700) != 0 && errno != EEXIST) return "";
    return d;
}

std::string cache_path(const std::string &dir, const std::string &key)
{
    char name[48];
    std::snprintf(name, sizeof name, "/%016" PRIx64 "%016" PRIx64 ".co", fnv1a(key, 0xcbf29ce484222325ull),
                  fnv1a(key, 0x84222325cbf29ce4ull));
    return dir + name;
}

// A cache file is the key, a NUL byte, then the code object.
bool cache_load(const std::string &path, const std::string &key, std::vector<char> &code)
{
    std::vector<char> all;
    if (!read_file(path, all) || all.size() <= key.size() + 1) return false;
    if (std::memcmp(all.data(), key.data(), key.size()) != 0 || all[key.size()] != '\0') return false;
    code.assign(all.begin() + key.size() + 1, all.end());
    return true;
}

// Written to a temporary name and renamed, so that readers see whole files.
void cache_store(const std::string &path, const std::string &key, const std::vector<char> &code)
{
    std::string tmp = path + ".XXXXXX";
    const int fd = mkstemp(&tmp[0]);
    if (fd < 0) return;
    bool ok = write(fd, key.data(), key.size()) == (ssize_t)key.size() && write(fd, "", 1) == 1 &&
              write(fd, code.data(), code.size()) == (ssize_t)code.size();
    ok = (close(fd) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) unlink(tmp.c_str());
}

// Compiles each source into a code object for `arch`: from the process
// cache, else the disk cache, else by the ROCm clang, the remaining sources
// in parallel child processes.
int compile(const std::vector<std::string> &srcs, const std::string &arch, std::vector<std::vector<char>> &codes)
{
    const std::string clang = rocm_path() + "/llvm/bin/clang++";
    // packed FP32 instructions are off for all device code of the library
    const std::vector<std::string> opts = {"-x", "hip", "--cuda-device-only", "--no-gpu-bundle-output",
                                           "--offload-arch=" + arch, "-O3", "-std=c++17", "-Xclang",
                                           "-target-feature", "-Xclang", "-packed-fp32-ops", "-w"};
    std::string common = clang + "\n";
    for (const auto &o : opts) common += o + "\n";
    for (int h = 0; h < kRtcNumHeaders; h++) common += std::string(kRtcHeaderNames[h]) + "\n" + kRtcHeaderSources[h];
    const size_t n = srcs.size();
    std::vector<std::string> keys(n);
    for (size_t k = 0; k < n; k++) keys[k] = common + "\n" + srcs[k];
    codes.assign(n, {});
    std::vector<size_t> todo;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (size_t k = 0; k < n; k++) {
            auto it = g_code.find(keys[k]);
            if (it != g_code.end()) codes[k] = it->second;
            else todo.push_back(k);
        }
    }
    const std::string cdir = todo.empty() ? "" : cache_dir();
    if (!cdir.empty()) {
        std::vector<size_t> left;
        for (size_t k : todo)
            if (!cache_load(cache_path(cdir, keys[k]), keys[k], codes[k])) left.push_back(k);
        todo.swap(left);
    }
    std::string err;
    if (!todo.empty()) {
        const char *tmp = std::getenv("TMPDIR");
        std::string dir = std::string(tmp && *tmp ? tmp : "/tmp") + "/qs_jit_XXXXXX";
        if (!mkdtemp(&dir[0])) return fail(QS_E_HIP, "cannot create a directory for run-time compilation");
        std::vector<std::string> files;
        for (int h = 0; h < kRtcNumHeaders; h++) {
            files.push_back(dir + "/" + kRtcHeaderNames[h]);
            write_file(files.back(), kRtcHeaderSources[h]);
        }
        std::vector<pid_t> pids(todo.size(), -1);
        for (size_t j = 0; j < todo.size(); j++) {
            const std::string base = dir + "/steps_" + std::to_string(todo[j]);
            files.insert(files.end(), {base + ".hip", base + ".co", base + ".log"});
            write_file(base + ".hip", srcs[todo[j]]);
            std::vector<std::string> args = {clang};
            args.insert(args.end(), opts.begin(), opts.end());
            args.insert(args.end(), {"-I" + dir, "-o", base + ".co", base + ".hip"});
            std::vector<char *> argv;
            for (auto &x : args) argv.push_back(&x[0]);
            argv.push_back(nullptr);
            posix_spawn_file_actions_t fa;
            posix_spawn_file_actions_init(&fa);
            posix_spawn_file_actions_addopen(&fa, 1, (base + ".log").c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
            posix_spawn_file_actions_adddup2(&fa, 1, 2);
            if (posix_spawn(&pids[j], clang.c_str(), &fa, nullptr, argv.data(), environ) != 0) {
                pids[j] = -1;
                err = "cannot start " + clang;
            }
            posix_spawn_file_actions_destroy(&fa);
        }
        for (size_t j = 0; j < todo.size(); j++) {
            if (pids[j] < 0) continue;
            int status = 0;
            while (waitpid(pids[j], &status, 0) < 0 && errno == EINTR) {
            }
            const size_t k = todo[j];
            const std::string base = dir + "/steps_" + std::to_string(k);
            if (!WIFEXITED(status) || WEXITSTATUS(status) != 0 || !read_file(base + ".co", codes[k]) ||
                codes[k].empty()) {
                std::vector<char> log;
                read_file(base + ".log", log);
                if (err.empty())
                    err = "run-time compilation of tile steps failed: " +
                          std::string(log.begin(), log.end()).substr(0, 2000);
            } else if (!cdir.empty()) {
                cache_store(cache_path(cdir, keys[k]), keys[k], codes[k]);
            }
        }
        for (const auto &f : files) unlink(f.c_str());
        rmdir(dir.c_str());
    }
    if (!err.empty()) return fail(QS_E_HIP, err);
    std::lock_guard<std::mutex> lock(g_mu);
    for (size_t k = 0; k < n; k++) g_code[keys[k]] = codes[k];
    return QS_OK;
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
    int rc = compile(specialized_sources(c, chunks, max_lds), arch, codes);
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
