// Run-time compilation of device code for the specialised tile steps and
// batch steps: HIP source -> code object for the current GPU, by the ROCm
// clang run as child processes, with a process cache and an on-disk cache.  (hiprtc is not
// used: in a process that has loaded PyTorch it resolves to the compiler
// bundled with PyTorch, whose code for these kernels spills to scratch
// memory.)
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
#include <cstring>
#include <fstream>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

// kRtcHeaderNames / kRtcHeaderSources: dev_core.hpp, tile_dev.hpp and
// batch_dev.hpp as strings (written by the build from the sources in this
// directory)
#include "qs_rtc_headers.inc"

extern char **environ;

namespace qs {

namespace {

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
// qs_jit_cache under $TMPDIR (default /tmp); empty (no disk cache) if it
// cannot be made or is not a directory of this user closed to others.
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
    // code objects are loaded from here: only a directory of this user that
    // no one else may write to
    struct stat sb;
    if (lstat(d.c_str(), &sb) != 0 || !S_ISDIR(sb.st_mode) || sb.st_uid != geteuid() || (sb.st_mode & 022) != 0)
        return "";
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

}  // namespace

// Compiles each source into a code object for `arch`: from the process
// cache, else the disk cache, else by the ROCm clang, the remaining sources
// in parallel child processes.
int compile_device_sources(const std::vector<std::string> &srcs, const std::string &arch,
                           std::vector<std::vector<char>> &codes)
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
                    err = "run-time compilation failed: " +
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

}  // namespace qs
