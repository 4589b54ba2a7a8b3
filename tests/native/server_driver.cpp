// Host-side checks of libfge's scheduler and planner, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (and, for the threaded part, ThreadSanitizer) by
// tests/test_sanitizers.py.  Everything here runs on the CPU: the server uses the simulated
// executor, the planner and parameter checks are host code.  Exits non-zero on a failed check;
// the sanitizers abort on a finding.
//
// usage: server_driver [manual|threaded|plan]...
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "fge.h"

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

namespace {

// Fake device addresses of request k (never dereferenced by the simulated executor).
void ptrs(int64_t k, void **I, void **A, void **F, void **B) {
    const uintptr_t base = static_cast<uintptr_t>(1) << 40;
    void **p[4] = {I, A, F, B};
    for (int i = 0; i < 4; ++i)
        *p[i] = reinterpret_cast<void *>(base + (static_cast<uintptr_t>(4 * k + i) << 32));
}

fge_status submit(fge_server *s, int64_t k, int H, int W) {
    void *I, *A, *F, *B;
    ptrs(k, &I, &A, &F, &B);
    return fge_server_submit(s, k, I, A, H, W, F, B);
}

int drain_results(fge_server *s, std::vector<fge_server_result> &out) {
    fge_server_result buf[64];
    int total = 0;
    for (;;) {
        const int n = fge_server_poll(s, buf, 64);
        if (n <= 0) return n < 0 && total == 0 ? n : total;
        out.insert(out.end(), buf, buf + n);
        total += n;
    }
}

void run_manual() {
    fge_params p;
    fge_default_params(&p);
    p.storage = FGE_F16;
    fge_server_config c;
    fge_server_default_config(&c);
    c.max_active = 7;
    c.budget_bytes = 3 * fge_server_request_bytes(1200, 1600, &p);
    for (int fail = 0; fail <= 2; ++fail) {
        fge_server_sim m;
        fge_server_sim_default(&m);
        if (fail == 1) m.fail_launch_tick = 5;
        if (fail == 2) m.fail_device_tick = 9;
        fge_server *s = nullptr;
        CHECK(fge_server_create_simulated(&p, &c, size_t(8) << 30, &m, &s) == FGE_OK);
        uint32_t rng = 12345;
        auto next = [&] { rng = rng * 1664525u + 1013904223u; return rng >> 8; };
        int submitted = 0;
        for (int k = 0; k < 150; ++k) {
            const int H = 1 + next() % 1200, W = 1 + next() % 1600;
            if (submit(s, k, H, W) == FGE_OK) ++submitted;
            if (k % 7 == 3) (void)fge_server_cancel(s, k - 1);
            if (k % 5 == 0) {
                const int32_t r = fge_server_sim_step(s, 1 + k % 3, 0.01 * k);
                CHECK(r >= 0 || fail == 2);
            }
        }
        (void)fge_server_drain(s);
        std::vector<fge_server_result> res;
        drain_results(s, res);
        CHECK(static_cast<int>(res.size()) == submitted);
        std::vector<int> seen(150, 0);
        for (const auto &r : res) {
            CHECK(r.id >= 0 && r.id < 150 && seen[r.id]++ == 0);
            CHECK(r.status == FGE_OK || r.status == FGE_ECANCELED || r.status == FGE_EHIP);
            if (fail == 0) CHECK(r.status != FGE_EHIP);
        }
        fge_server_stats st;
        CHECK(fge_server_get_stats(s, &st) == FGE_OK);
        CHECK(st.peak_charged_bytes <= c.budget_bytes && st.peak_active <= 7);
        CHECK(st.completed == submitted);
        fge_server_destroy(s);
    }
    std::printf("manual: ok\n");
}

void run_threaded() {
    fge_params p;
    fge_default_params(&p);
    fge_server_config c;
    fge_server_default_config(&c);
    c.max_active = 12;
    fge_server_sim m;
    fge_server_sim_default(&m);
    m.manual = 0;
    m.us_per_launch = 1.0;
    m.us_per_mpx = 1.0;
    fge_server *s = nullptr;
    CHECK(fge_server_create_simulated(&p, &c, size_t(16) << 30, &m, &s) == FGE_OK);
    const int per = 60, nthreads = 4;
    std::atomic<int> ok{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
        th.emplace_back([&, t] {
            for (int i = 0; i < per; ++i) {
                const int64_t k = t * per + i;
                if (submit(s, k, 1 + (k * 37) % 1100, 1 + (k * 53) % 900) == FGE_OK) ++ok;
                if (i % 9 == 4) (void)fge_server_cancel(s, k);
            }
        });
    std::vector<fge_server_result> res;
    std::thread poller([&] {
        while (static_cast<int>(res.size()) < nthreads * per) {
            fge_server_result buf[32];
            const int n = fge_server_poll(s, buf, 32);
            if (n > 0) res.insert(res.end(), buf, buf + n);
            else std::this_thread::yield();
        }
    });
    for (auto &x : th) x.join();
    CHECK(fge_server_drain(s) == FGE_OK);
    poller.join();
    CHECK(ok.load() == nthreads * per);
    std::vector<int> seen(nthreads * per, 0);
    for (const auto &r : res) {
        CHECK(seen[r.id]++ == 0);
        CHECK(r.status == FGE_OK || r.status == FGE_ECANCELED);
    }
    fge_server_stats st;
    CHECK(fge_server_get_stats(s, &st) == FGE_OK && st.completed == nthreads * per);
    fge_server_destroy(s);
    std::printf("threaded: ok\n");
}

void run_plan() {
    fge_params p;
    fge_default_params(&p);
    int32_t w[16], h[16], it[16], n = 0, nc = 0;
    for (int H = 1; H <= 3000; H += 37)
        for (int W = 1; W <= 3000; W += 41) {
            for (int storage = 0; storage < 2; ++storage) {
                p.storage = storage;
                CHECK(fge_plan(H, W, &p, 16, w, h, it, &n, &nc) == FGE_OK);
                CHECK(n >= 1 && n <= 16 && nc >= 0 && nc <= n && w[n - 1] == W && h[n - 1] == H);
                (void)fge_workspace_bytes(H, W, &p);
                (void)fge_server_request_bytes(H, W, &p);
            }
        }
    CHECK(fge_plan(0, 5, &p, 16, w, h, it, &n, &nc) == FGE_EINVAL);
    CHECK(fge_plan(40000, 5, &p, 16, w, h, it, &n, &nc) == FGE_EINVAL);
    CHECK(fge_plan(32767, 32767, &p, 16, w, h, it, &n, &nc) == FGE_OK);
    // closed-form argument checks return before any device call
    fge_cf_params cp;
    fge_cf_default_params(&cp);
    CHECK(fge_cf_workspace_bytes(768, 1024) > 0);
    CHECK(fge_closed_form(nullptr, nullptr, 1, 1, &cp, nullptr, nullptr, nullptr, 0, nullptr,
                          nullptr) == FGE_EINVAL);
    std::printf("plan: ok\n");
}

}  // namespace

int main(int argc, char **argv) {
    for (int i = 1; i < argc; ++i) {
        if (!std::strcmp(argv[i], "manual")) run_manual();
        else if (!std::strcmp(argv[i], "threaded")) run_threaded();
        else if (!std::strcmp(argv[i], "plan")) run_plan();
        else return 2;
    }
    return 0;
}
