// Tuning knobs of the launch policy.  Defaults come from measurements on
// MI355X; the environment can override them (QS_DENSE_KERNEL=vector|mfma,
// QS_MFMA_BLOCKS=<max blocks of the MFMA kernel>).
#include "common.hpp"

#include <cstdlib>

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

uint64_t mfma_block_cap(int)
{
    static const uint64_t cap = [] {
        const char *e = std::getenv("QS_MFMA_BLOCKS");
        if (e) {
            const unsigned long long v = std::strtoull(e, nullptr, 10);
            if (v > 0) return (uint64_t)v;
        }
        return (uint64_t)1 << 30;
    }();
    return cap;
}

}  // namespace qs
