// Host-only driver for the C ABI's plan code (validation, static orders, bit
// packing, root classes, workspace layout), built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the CPU.  The search kernels are stubbed out:
// nothing here launches device code; without a GPU the HIP queries fail and
// the plan falls back to its default launch shape.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mcs.h"

static char g_dummy_kernel;
extern "C" void *mcs_internal_search_kernel(int, int, int) { return &g_dummy_kernel; }
extern "C" void *mcs_internal_reset_kernel(void) { return &g_dummy_kernel; }
extern "C" void *mcs_internal_seg_kernel(int, int, int) { return &g_dummy_kernel; }
extern "C" void *mcs_internal_static_scratch(size_t *bytes, int *err) {
    *bytes = 0;
    *err = -1;  // no device here
    return nullptr;
}

static uint64_t g_state = 0x1234567ull;
static uint64_t next_u64() {  // splitmix64
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Graph {
    int n = 0, directed = 0;
    std::vector<uint64_t> adj;
    std::vector<int32_t> label;
    bool labelled = false;
    mcs_graph view() const {
        static const int32_t none = 0;  // (a labelled graph of no vertices)
        mcs_graph g{};
        g.n = n;
        g.directed = directed;
        g.adj = adj.empty() ? nullptr : adj.data();
        g.label = !labelled ? nullptr : label.empty() ? &none : label.data();
        return g;
    }
};

static Graph random_graph(int n, double p, int directed, int labels) {
    Graph g;
    g.n = n;
    g.directed = directed;
    const int rw = n <= 64 ? 1 : (n + 63) / 64;
    g.adj.assign((size_t)(n > 0 ? n : 1) * rw, 0);
    auto set = [&](int i, int j) { g.adj[(size_t)i * rw + j / 64] |= 1ull << (j % 64); };
    for (int i = 0; i < n; i++)
        for (int j = directed ? 0 : i + 1; j < n; j++) {
            if (i == j)
                continue;
            if ((double)(next_u64() >> 11) * 0x1.0p-53 < p) {
                set(i, j);
                if (!directed)
                    set(j, i);
            }
        }
    g.labelled = labels > 0;
    if (labels > 0)
        for (int i = 0; i < n; i++)
            g.label.push_back((int32_t)(next_u64() % (uint64_t)labels));
    return g;
}

static int failures = 0;
static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, mcs_last_error());
        failures++;
    }
}

int main() {
    const int sizes[] = {1, 16, 33, 64, 65, 100, 128, 129, 193, 254};
    for (int ordering = 0; ordering < 2; ordering++)
        for (int directed = 0; directed < 2; directed++)
            for (int labels : {0, 3, 70})
                for (int a : sizes) {
                    std::vector<Graph> Gs, Hs;
                    for (int b : sizes) {
                        Gs.push_back(random_graph(a, 0.2, directed, labels));
                        Hs.push_back(random_graph(b, 0.3, directed, labels));
                    }
                    Gs.push_back(random_graph(0, 0.0, directed, labels));
                    Hs.push_back(random_graph(a, 0.5, directed, labels));
                    std::vector<mcs_graph> G, H;
                    for (size_t i = 0; i < Gs.size(); i++) {
                        G.push_back(Gs[i].view());
                        H.push_back(Hs[i].view());
                    }
                    mcs_opts o{};
                    o.ordering = ordering;
                    mcs_plan *p = nullptr;
                    expect(mcs_plan_create((int32_t)G.size(), G.data(), H.data(), &o, &p) ==
                               MCS_OK,
                           "plan create");
                    if (p) {
                        std::vector<int32_t> rb(G.size());
                        expect(mcs_plan_root_bounds(p, rb.data()) == MCS_OK, "root bounds");
                        for (size_t i = 0; i < G.size(); i++)
                            expect(rb[i] >= 0 && rb[i] <= MCS_MAX_N, "root bound range");
                        mcs_plan_destroy(p);
                    }
                    expect(mcs_workspace_size((int32_t)G.size(), G.data(), H.data(), &o) > 0,
                           "workspace size");
                }
    // rejected inputs: a bit at or above n in the second word, a self loop in
    // the second word, an asymmetric undirected graph, too many vertices
    // (255: the limit is 254)
    {
        Graph g = random_graph(100, 0.2, 0, 0), h = random_graph(100, 0.2, 0, 0);
        mcs_graph G = g.view(), H = h.view();
        mcs_plan *p = nullptr;
        g.adj[2 * 5 + 1] |= 1ull << 40;  // vertex 104 of row 5
        G = g.view();
        expect(mcs_plan_create(1, &G, &H, nullptr, &p) == MCS_E_INVALID, "bit above n");
        g = random_graph(100, 0.2, 0, 0);
        g.adj[2 * 90 + 1] |= 1ull << (90 - 64);
        G = g.view();
        expect(mcs_plan_create(1, &G, &H, nullptr, &p) == MCS_E_INVALID, "self loop");
        g = random_graph(100, 0.2, 0, 0);
        g.adj[2 * 3 + 1] ^= 1ull << (80 - 64);
        G = g.view();
        expect(mcs_plan_create(1, &G, &H, nullptr, &p) == MCS_E_INVALID, "asymmetric");
        Graph big = random_graph(MCS_MAX_N + 1, 0.1, 1, 0);
        G = big.view();
        expect(mcs_plan_create(1, &G, &H, nullptr, &p) == MCS_E_TOO_LARGE, "too large");
    }
    std::printf("%s\n", failures ? "host plan checks failed" : "host plan checks passed");
    return failures ? 1 : 0;
}
