// Exercises the host-side paths of libpitsbicg that need no GPU (context
// creation and validation, the line/column/velocity/per-slice table
// builders, workspace sizing, the autotuner's candidate sizing, batch engine
// creation) and the request server's arena allocator, for a build of the
// library's host code with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  No HIP call is made.  Exit 0 when every
// check held; the sanitizers abort on a fault.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "arena.hpp"
#include "pitsbicg.h"

namespace {

int failures = 0;
void check(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

pit_problem problem(int dim, int Mx, int My, int bc, double nu, double ax, double rot, double react)
{
    pit_problem p{};
    p.dim = dim;
    p.M[0] = Mx;
    p.M[1] = My;
    p.bc = bc;
    p.length[0] = 1.0;
    p.length[1] = 1.0;
    p.nu = nu;
    p.adv[0] = ax;
    p.adv[1] = 0.0;
    p.react = react;
    p.T = 0.5;
    p.rot = rot;
    return p;
}

// Random allocations and releases against a model of the live ranges: no
// two live ranges overlap, every range lies inside the arena, the used
// count matches, and freeing everything leaves one free range.
void arena_test()
{
    const size_t base = 4096, size = 256 * 1000;
    pit::Arena a;
    a.init(base, size);
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> live;  // offset, requested bytes
    size_t used = 0;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = 1 + rng() % 9000;
            size_t off = 0;
            if (a.alloc(want, off)) {
                const size_t r = pit::arena_round(want);
                check(off >= base && off + r <= base + size, "arena range inside the arena");
                check(off % pit::kArenaAlign == 0, "arena offset aligned");
                for (const auto &l : live) {
                    const size_t lr = pit::arena_round(l.second);
                    check(off + r <= l.first || l.first + lr <= off, "arena ranges disjoint");
                }
                live.emplace_back(off, want);
                used += r;
            } else {
                check(a.largest() < pit::arena_round(want), "arena refuses only what does not fit");
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].first, live[i].second);
            used -= pit::arena_round(live[i].second);
            live.erase(live.begin() + (long)i);
        }
        check(a.used == used, "arena used count");
    }
    for (const auto &l : live) a.release(l.first, l.second);
    check(a.used == 0 && a.free.size() == 1 && a.largest() == size, "arena coalesces back to one range");
}

void contexts()
{
    const pit_stepper ie{PIT_IE, 0, PIT_F64, 0}, cn{PIT_CN, 0, PIT_F64, 0}, cn32{PIT_CN, 0, PIT_F32, 0};
    const pit_stepper ie2{PIT_IE, 2, PIT_F64, 0}, adi{PIT_ADI_PR, 0, PIT_F64, 0}, adi32{PIT_ADI_PR, 0, PIT_F32, 0};
    const pit_stepper adic{PIT_ADI_PR, 1, PIT_F64, 0}, adiie{PIT_ADI_IE, 1, PIT_F64, 0};
    struct Case {
        pit_problem p;
        int N, m;
        pit_stepper f, g;
    };
    std::vector<Case> ok = {
        {problem(1, 64, 1, PIT_DIRICHLET0, 0.1, 0, 0, 0), 16, 64, ie, {PIT_IE, 1, PIT_F64, 0}},
        {problem(1, 1000, 1, PIT_PERIODIC, 1e-3, 1.0, 0, 0.2), 12, 20, cn, ie2},
        {problem(1, 4096, 1, PIT_PERIODIC, 1e-3, 1.0, 0, 0), 8, 10, cn32, ie2},
        {problem(1, 12000, 1, PIT_PERIODIC, 1e-3, 1.0, 0, 0), 4, 3, cn, ie2},
        {problem(1, 3, 1, PIT_DIRICHLET0, 0.1, 0, 0, 0), 3, 2, ie, {PIT_IE, 1, PIT_F64, 0}},
        {problem(2, 40, 33, PIT_DIRICHLET0, 0.05, 0, 0, 0.2), 4, 3, adi, adic},
        {problem(2, 512, 512, PIT_DIRICHLET0, 0.05, 0, 0, 0), 8, 4, adi32, adic},
        {problem(2, 700, 130, PIT_DIRICHLET0, 0.05, 0, 0, 0), 3, 2, adi32, adic},
        {problem(2, 49, 49, PIT_DIRICHLET0, 0.1, 0, 1.0, 0.5), 8, 5, adi, adic},
        {problem(2, 160, 150, PIT_DIRICHLET0, 0.1, 0.2, 1.0, 0.5), 4, 3, adi, adiie},
    };
    for (auto &c : ok) {
        pit_ctx *h = nullptr;
        check(pit_create(&c.p, c.N, c.m, c.f, c.g, &h) == PIT_OK && h, "pit_create accepts a valid problem");
        if (!h) continue;
        const size_t base = pit_workspace_bytes(h);
        int32_t shape[4];
        check(pit_kernel_shape(h, shape) == PIT_OK, "pit_kernel_shape");
        std::vector<double> f((size_t)c.p.M[0] * (c.p.dim == 2 ? c.p.M[1] : 1), 0.25);
        std::vector<double> g((size_t)c.N * c.m + 1, 1.5);
        check(pit_set_source(h, f.data()) == PIT_OK, "pit_set_source unbound");
        check(pit_set_source_t(h, f.data(), g.data()) == PIT_OK && pit_workspace_bytes(h) > base,
              "pit_set_source_t grows the workspace");
        check(pit_set_source(h, nullptr) == PIT_OK && pit_workspace_bytes(h) == base, "source removed");
        std::vector<double> s((size_t)c.N);
        for (int n = 0; n < c.N; ++n) s[(size_t)n] = 0.5 + 0.3 * n;
        const int rc = pit_set_nu_t(h, s.data());
        check(c.p.dim == 2 ? rc == PIT_EINVAL : (rc == PIT_OK && pit_workspace_bytes(h) > base),
              "pit_set_nu_t: 1D grows the workspace, 2D refused");
        check(pit_set_nu_t(h, nullptr) == PIT_OK && pit_workspace_bytes(h) == base, "per-slice operator removed");
        const size_t tune = pit_autotune_scratch_bytes(&c.p, c.N, c.m, c.f, c.g);  // 0: nothing to tune
        check(tune == 0 || tune >= base, "autotune scratch covers the context");
        check(pit_apply_F(h, nullptr, nullptr, 0, nullptr) == PIT_EINVAL, "unbound apply refused");
        check(pit_destroy(h) == PIT_OK, "pit_destroy");
    }
    // refused descriptions
    pit_ctx *h = nullptr;
    pit_problem bad = problem(1, 2, 1, PIT_DIRICHLET0, 0.1, 0, 0, 0);
    check(pit_create(&bad, 4, 4, ie, ie, &h) == PIT_EINVAL && !h, "M < 3 refused");
    bad = problem(1, 64, 1, PIT_DIRICHLET0, -1.0, 0, 0, 0);
    check(pit_create(&bad, 4, 4, ie, ie, &h) == PIT_EINVAL, "negative nu refused");
    bad = problem(2, 64, 64, PIT_PERIODIC, 0.1, 0, 0, 0);
    check(pit_create(&bad, 4, 4, adi, adic, &h) == PIT_EINVAL, "periodic 2D refused");
    bad = problem(2, 64, 64, PIT_DIRICHLET0, 0.1, 0, 1.0, 0);
    check(pit_create(&bad, 4, 4, adi32, adic, &h) == PIT_EINVAL, "FP32 with a velocity field refused");
    bad = problem(1, 64, 1, PIT_DIRICHLET0, 0.1, 0, 0, 0);
    check(pit_create(&bad, 0, 4, ie, ie, &h) == PIT_EINVAL, "N < 1 refused");
    for (int code : {PIT_OK, PIT_EINVAL, PIT_ENOMEM, PIT_EHIP, PIT_ENOCONV, PIT_EBREAKDOWN, PIT_EAGAIN, 12345})
        check(pit_strerror(code) != nullptr, "pit_strerror");
    pit_batch *b = nullptr;
    check(pit_batch_create(64, &b) == PIT_OK && b && pit_batch_workspace_bytes(b) > 0, "batch engine");
    check(pit_batch_destroy(b) == PIT_OK, "batch engine destroyed");
}

}  // namespace

int main()
{
    arena_test();
    contexts();
    std::printf("host driver: %s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
