// Launch-policy knobs and the fusion-width autotuner.
//
// Knobs default to values measured on MI355X and can be overridden from the
// environment: QS_DENSE_KERNEL=vector|mfma (dense gates of 4-6 targets on
// complex64), QS_MFMA_BLOCKS=<max blocks of the MFMA kernel>,
// QS_TILE_LOW=<lowest qubits every tile step holds>,
// QS_STEP_WAVES=<waves per SIMD the specialised tile steps are compiled for>,
// QS_TILE_CHUNK=<tiles per block of the chunk policy; unset: as many blocks
// as stay resident>, QS_TILE_GRID=chunk|stride|tiles (tile-step grids: resident blocks each
// walking a run of consecutive tiles, resident blocks walking by a fixed
// stride, or one block per tile; by default one block per tile for tiles of
// up to 2^12 amplitudes and a stride for larger ones).
#include "common.hpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

namespace qs {

int mfma_preference()
{
    static const int pref = [] {
        const char *e = std::getenv("QS_DENSE_KERNEL");
        if (e && std::string(e) == "vector") return 0;
        return 1;
    }();
    return pref;
}

uint64_t mfma_block_cap(int k)
{
    static const uint64_t forced = [] {
        const char *e = std::getenv("QS_MFMA_BLOCKS");
        if (e) {
            const unsigned long long v = std::strtoull(e, nullptr, 10);
            if (v > 0) return (uint64_t)v;
        }
        return (uint64_t)0;
    }();
    if (forced) return forced;
    // measured on MI355X at 28 qubits: one tile per wave is best for 4
    // targets; 5 and 6 targets do better with waves that walk several tiles
    // (the 16-64 KiB A operand is staged into LDS once per block)
    if (k >= 6) return 2048;
    if (k == 5) return 8192;
    return (uint64_t)1 << 30;
}

int step_waves_per_eu(bool f32)
{
    static const int forced = [] {
        const char *e = std::getenv("QS_STEP_WAVES");
        if (e) {
            const int v = std::atoi(e);
            if (v >= 1 && v <= 8) return v;
        }
        return 0;
    }();
    if (forced) return forced;
    return f32 ? 6 : 4;
}

uint64_t tile_chunk()
{
    static const uint64_t v = [] {
        const char *e = std::getenv("QS_TILE_CHUNK");
        if (e) {
            const unsigned long long k = std::strtoull(e, nullptr, 10);
            if (k >= 1 && k <= (1ull << 20)) return (uint64_t)k;
        }
        return (uint64_t)0;
    }();
    return v;
}

int tile_grid_policy(int tile_d)
{
    static const int forced = [] {
        const char *e = std::getenv("QS_TILE_GRID");
        if (e && std::string(e) == "stride") return (int)kTileGridStride;
        if (e && std::string(e) == "tiles") return (int)kTileGridPerTile;
        if (e && std::string(e) == "chunk") return (int)kTileGridChunk;
        return -1;
    }();
    if (forced >= 0) return forced;
    // measured on the 28-qubit random circuit (complex64, specialised steps):
    // one block per tile is best for tiles of up to 2^12 amplitudes (2^12:
    // 55.1 ms against 60.0 ms striding); 2^13-amplitude tiles (1024-thread
    // blocks) keep resident blocks striding (52.5 ms against 56.7 ms)
    return tile_d >= 13 ? kTileGridStride : kTileGridPerTile;
}

int tile_low_qubits(int precision)
{
    static const int forced = [] {
        const char *e = std::getenv("QS_TILE_LOW");
        if (e) {
            const int v = std::atoi(e);
            if (v >= 1 && v <= 8) return v;
        }
        return 0;
    }();
    if (forced) return forced;
    return precision == QS_C64 ? 4 : 3;   // 128-byte runs
}

// (qubits, precision (+4 when specialised steps were candidates), circuit
// fingerprint) -> chosen fusion width, with kSpecialisedFlag set when the
// tile steps run specialised
using TuneKey = std::tuple<int, int, uint64_t>;
static std::map<TuneKey, int> g_tuned;
static std::mutex g_tune_mu;
static bool g_file_loaded = false;

static void load_cache_file()
{
    if (g_file_loaded) return;
    g_file_loaded = true;
    const char *path = std::getenv("QS_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int n, p, k;
    unsigned long long h;
    while (std::fscanf(f, "fuse %d %d %llx %d\n", &n, &p, &h, &k) == 4) g_tuned[TuneKey(n, p, h)] = k;
    std::fclose(f);
}

static void append_cache_file(const TuneKey &key, int k)
{
    const char *path = std::getenv("QS_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "fuse %d %d %llx %d\n", std::get<0>(key), std::get<1>(key),
                 (unsigned long long)std::get<2>(key), k);
    std::fclose(f);
}

}  // namespace qs

using namespace qs;

namespace {

// A tuned choice: fusion width k, and whether the tile steps run as
// specialised kernels (stored as k + kSpecialisedFlag).
constexpr int kSpecialisedFlag = 1 << 16;

// Applies the circuit once untimed (first touch, code loading) and once
// between two events on q's stream; *ms receives the timed application.
int time_application(qs_qureg *q, qs_circuit *c, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    int rc = qs_apply_circuit(q, c);
    if (rc != QS_OK) return rc;
    if (hipEventRecord(e0, q->stream) != hipSuccess) return fail(QS_E_HIP, "hipEventRecord");
    rc = qs_apply_circuit(q, c);
    if (rc != QS_OK) return rc;
    if (hipEventRecord(e1, q->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(QS_E_HIP, "event timing failed");
    *ms = 0.f;
    (void)hipEventElapsedTime(ms, e0, e1);
    return QS_OK;
}

// Leaves the circuit compiled (and specialised) as `choice` says.
int apply_choice(qs_circuit *c, int choice, int precision)
{
    int rc = qs_circuit_compile(c, choice & (kSpecialisedFlag - 1), precision);
    if (rc == QS_OK && (choice & kSpecialisedFlag)) rc = qs_circuit_specialize(c, nullptr);
    return rc;
}

}  // namespace

extern "C" int qs_circuit_autotune_ex(qs_qureg *q, qs_circuit *c, const int *candidates, int num_candidates,
                                      int try_specialized, int *best_k, int *best_specialized, double *ms_out,
                                      double *ms_specialized_out)
{
    if (!q || !c || !candidates || num_candidates < 1) return fail(QS_E_ARG, "bad autotune arguments");
    if (q->num_qubits != circuit_num_qubits(c)) return fail(QS_E_ARG, "qubit counts differ");
    const TuneKey key(q->num_qubits, q->precision + (try_specialized ? 4 : 0), circuit_fingerprint(c));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_file();
        auto it = g_tuned.find(key);
        if (it != g_tuned.end() && !ms_out && !ms_specialized_out) {
            if (best_k) *best_k = it->second & (kSpecialisedFlag - 1);
            if (best_specialized) *best_specialized = (it->second & kSpecialisedFlag) != 0;
            return apply_choice(c, it->second, q->precision);
        }
    }
    hipEvent_t e0, e1;
    QS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(QS_E_HIP, "hipEventCreate");
    }
    int best = candidates[0];
    float best_ms = 1e30f;
    int rc = QS_OK;
    for (int i = 0; i < num_candidates && rc == QS_OK; i++) {
        if (ms_specialized_out) ms_specialized_out[i] = -1.0;
        rc = qs_circuit_compile(c, candidates[i], q->precision);
        if (rc != QS_OK) break;
        float ms = 0.f;
        rc = time_application(q, c, e0, e1, &ms);
        if (rc != QS_OK) break;
        if (ms_out) ms_out[i] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = candidates[i];
        }
        if (!try_specialized) continue;
        int kernels = 0;
        if (qs_circuit_specialize(c, &kernels) != QS_OK || kernels == 0) continue;   // no tile steps, or no compiler
        rc = time_application(q, c, e0, e1, &ms);
        if (rc != QS_OK) break;
        if (ms_specialized_out) ms_specialized_out[i] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = candidates[i] | kSpecialisedFlag;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != QS_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
        append_cache_file(key, best);
    }
    if (best_k) *best_k = best & (kSpecialisedFlag - 1);
    if (best_specialized) *best_specialized = (best & kSpecialisedFlag) != 0;
    return apply_choice(c, best, q->precision);
}

extern "C" int qs_circuit_autotune(qs_qureg *q, qs_circuit *c, const int *candidates, int num_candidates,
                                   int *best_k, double *ms_out)
{
    return qs_circuit_autotune_ex(q, c, candidates, num_candidates, 0, best_k, nullptr, ms_out, nullptr);
}
