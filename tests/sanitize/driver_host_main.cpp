// Exercises the library's host-only logic under AddressSanitizer / UndefinedBehaviorSanitizer
// (no device work): the extension plan of Alg. 2 over many sizes and leaf cutoffs, the
// workspace query over ragged batches (with plan merging, chunking and several streams),
// option validation (valid, invalid, boundary values), the error strings, launch timing with
// nothing launched and the prepared-batch calls' argument checks.
#include <cstdio>
#include <cstdint>
#include <vector>
#include "../../include/tikh.h"

int main() {
    int bad = 0;
    for (int64_t m = 1; m <= 3000; m += 37)
        for (int64_t n = 1; n <= 3000; n += 53)
            for (int32_t nlim : {64, 128, 192, 256}) {
                int64_t N = 0, M = 0, k = 0;
                int32_t p = 0;
                if (tikh_plan_info(m, n, nlim, &N, &M, &p, &k) != TIKH_OK) { bad = 1; continue; }
                if (N != ((int64_t)1 << p) * M || k != N - (m + n - 1) || k < 0) bad = 1;
            }
    tikh_opts o{};
    bad |= tikh_get_options(&o) != TIKH_OK;
    const tikh_opts keep = o;
    for (int chunk : {0, 1, 7}) {
        o = keep;
        o.chunk_groups = chunk;
        o.streams = chunk == 7 ? 1 : 16;
        bad |= tikh_set_options(&o) != TIKH_OK;
        std::vector<int64_t> ms, ns;
        for (int q = 0; q < 40; ++q) { ms.push_back(50 + 97 * q); ns.push_back(40 + 61 * q); }
        size_t bytes = 0;
        bad |= tikh_workspace_bytes((int64_t)ms.size(), ms.data(), ns.data(), 8, 4, &bytes) != TIKH_OK;
        bad |= bytes == 0;
        bad |= tikh_workspace_bytes(0, nullptr, nullptr, 1, 1, &bytes) != TIKH_OK || bytes != 0;
        int64_t zero = 0;
        bad |= tikh_workspace_bytes(1, &zero, &zero, 1, 1, &bytes) != TIKH_EINVAL;
    }
    o = keep;
    o.n_lim = 32;
    bad |= tikh_set_options(&o) != TIKH_EINVAL;
    o = keep;
    o.merge_tol = -1.0;
    bad |= tikh_set_options(&o) != TIKH_EINVAL;
    o = keep;
    o.refine_skip = 2;
    bad |= tikh_set_options(&o) != TIKH_EINVAL;
    bad |= tikh_set_options(&keep) != TIKH_OK;
    for (int code = 0; code >= -6; --code) bad |= tikh_strerror(code) == nullptr;
    // launch timing with nothing launched, and the prepared-batch calls' argument checks
    double ms = -1.0, units = -1.0;
    int64_t count = -1;
    bad |= tikh_profile_kernel("fft") != TIKH_OK;
    bad |= tikh_profile_read(&ms, &count) != TIKH_OK || ms != 0.0 || count != 0;
    bad |= tikh_profile_units(&units) != TIKH_OK || units != 0.0;
    bad |= tikh_profile_kernel(nullptr) != TIKH_OK;
    bad |= tikh_profile_read(nullptr, &count) != TIKH_EINVAL;
    size_t pbytes = 0;
    bad |= tikh_prepared_run(nullptr) != TIKH_EINVAL;
    bad |= tikh_prepared_workspace(nullptr, &pbytes) != TIKH_EINVAL;
    bad |= tikh_prepared_free(nullptr) != TIKH_OK;
    tikh_prepared* h = reinterpret_cast<tikh_prepared*>(1);
    int64_t pm = 8, pn = 8;
    double lam = 1.0;
    bad |= tikh_prepare_batched(1, &pm, &pn, nullptr, nullptr, 1, &lam, 1, nullptr, nullptr, nullptr, 0, &h) !=
           TIKH_EINVAL;
    bad |= h != nullptr;
    std::printf(bad ? "driver host sanitizer run: FAILED\n" : "driver host sanitizer run: clean\n");
    return bad;
}
