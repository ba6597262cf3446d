// Host-side driver for the sanitizer build of the library (AddressSanitizer and UndefinedBehavior-
// Sanitizer on the host code only; the device code is not built).  It exercises what runs without a
// GPU: every workspace query (a dry run of the solve, setup, batch, ladder and eigensolver paths with
// allocations counted) over shapes and options, option validation, and the batch planner called from
// four host threads at once (each result compared with the single-threaded one).  Exit status 0 when
// every query behaved; the sanitizers abort the process on the first memory or UB error.
#include "adc3ea.h"

#include <cstdio>
#include <thread>
#include <vector>

namespace {
struct Shape {
    int o, v, X, nr;
};
const Shape kShapes[] = {{4, 20, 60, 3}, {20, 200, 600, 5}, {3, 7, 15, 2}, {1, 1, 1, 1}, {40, 600, 1800, 5},
                         {30, 400, 1200, 5}, {6, 41, 60, 7}};

std::vector<adc3_instance> ragged(int n, int seed) {
    std::vector<adc3_instance> v;
    unsigned s = 12345u + 77u * seed;
    for (int i = 0; i < n; ++i) {
        s = s * 1103515245u + 12345u;
        adc3_instance in{};
        in.nocc = 2 + (s >> 8) % 12;
        in.nvir = 8 + (s >> 12) % 60;
        in.naux = 3 * in.nvir;
        in.nroots = 1 + (s >> 20) % 6;
        in.fno_thresh = (i % 3 == 0) ? 1e-4 : 0.0;
        in.naf_thresh = (i % 3 == 0) ? 1e-2 : 0.0;
        in.conv = 1e-6;
        v.push_back(in);
    }
    return v;
}
}  // namespace

int main() {
    int bad = 0;
    adc3_opts o;
    adc3_default_opts(&o);
    for (const Shape& sh : kShapes)
        for (int lock = -1; lock < 3; ++lock)
            for (int prec = 0; prec < 3; ++prec)
                for (int mode = 0; mode < 2; ++mode) {
                    adc3_opts p = o;
                    p.lockstep = lock;
                    p.precision = prec;
                    p.fno_mode = mode;
                    p.sm_x = 0.5;
                    if (adc3_ea_solve_workspace_bytes(sh.o, sh.v, sh.X, sh.nr, &p) == 0) {
                        std::printf("solve plan failed: o=%d v=%d X=%d lock=%d prec=%d mode=%d\n", sh.o, sh.v, sh.X,
                                    lock, prec, mode);
                        ++bad;
                    }
                    for (int level = 2; level <= 3; ++level)
                        if (adc3_ea_setup_workspace_bytes_ex(sh.o, sh.v, sh.X, level, sh.nr, prec, 0) == 0) ++bad;
                }
    // invalid options and sizes are refused with 0
    adc3_opts q = o;
    q.sm_x = 2.0;
    bad += adc3_ea_solve_workspace_bytes(4, 20, 60, 3, &q) != 0;
    q = o;
    q.fno_keep_frac = -1.0;
    bad += adc3_ea_solve_workspace_bytes(4, 20, 60, 3, &q) != 0;
    bad += adc3_ea_solve_workspace_bytes(0, 20, 60, 3, &o) != 0;
    bad += adc3_ea_setup_workspace_bytes_ex(4, 20, 60, 4, 3, 0, 0) != 0;
    bad += adc3_ladder_workspace_bytes(600, 1800, 200, 2) == 0;
    bad += adc3_eigh_workspace_bytes(200) == 0;
    bad += adc3_eigh_batched_workspace_bytes(96, 5) == 0;
    // the batch planner from four threads at once, each checked against the single-threaded answer
    std::vector<std::vector<adc3_instance>> sets;
    std::vector<size_t> ref;
    for (int t = 0; t < 4; ++t) {
        sets.push_back(ragged(9 + t, t));
        adc3_opts p = o;
        p.lockstep = t % 3;
        ref.push_back(adc3_ea_solve_batched_workspace_bytes(sets[t].data(), (int)sets[t].size(), &p, 1 + t));
        if (ref[t] == 0) ++bad;
    }
    std::vector<size_t> got(4, 0);
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
        th.emplace_back([&, t] {
            adc3_opts p = o;
            p.lockstep = t % 3;
            for (int rep = 0; rep < 3; ++rep)
                got[t] = adc3_ea_solve_batched_workspace_bytes(sets[t].data(), (int)sets[t].size(), &p, 1 + t);
        });
    for (auto& x : th) x.join();
    for (int t = 0; t < 4; ++t)
        if (got[t] != ref[t]) {
            std::printf("thread %d: %zu != %zu\n", t, got[t], ref[t]);
            ++bad;
        }
    std::printf("plan driver: %d problems\n", bad);
    return bad == 0 ? 0 : 1;
}
