// Host side of the C ABI declared in include/mcs.h: validation, degree
// ordering and bit packing, workspace layout, kernel launches (direct or from
// a HIP graph), and mapping the results back to the caller's vertex ids.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mcs.h"
#include "mcs_layout.h"

extern "C" void *mcs_internal_search_kernel(int word_bytes, int directed, int policy);
extern "C" void *mcs_internal_seg_kernel(int word_bytes, int directed, int seg_log);
extern "C" void *mcs_internal_static_scratch(size_t *bytes, int *err);
extern "C" void *mcs_internal_reset_kernel(void);

// LDS allocation granule assumed for gfx950 workgroups (bytes): a multiple
// of the hardware's unit, so that counting in it never over-commits a CU.
static constexpr int kLdsGranule = 2048;

namespace {

thread_local std::string g_err;

mcs_status fail(mcs_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

mcs_status hip_fail(hipError_t e, const char *what) {
    return fail(MCS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                              \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess)                      \
            return hip_fail(e_, #call);            \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint64_t low_mask(int n) { return n >= 64 ? ~0ull : n <= 0 ? 0ull : ((1ull << n) - 1); }

// 64-bit words per adjacency row of the caller's graph: one up to 64
// vertices, then one more per 64 vertices.
int row_words(int n) { return n <= 64 ? 1 : (n + 63) / 64; }

// Arc i -> j of the caller's graph (bit j % 64 of word j / 64 of row i).
bool in_arc(const mcs_graph &g, int i, int j) {
    return (g.adj[(size_t)i * row_words(g.n) + (j >> 6)] >> (j & 63)) & 1;
}

// A vertex set (a row or one side of a class) of up to 256 vertices.
struct Bits {
    uint64_t w[4] = {0, 0, 0, 0};
    void set(int j) { w[j >> 6] |= 1ull << (j & 63); }
    bool get(int j) const { return (w[j >> 6] >> (j & 63)) & 1; }
    bool any() const { return (w[0] | w[1] | w[2] | w[3]) != 0; }
};

Bits first_n(int n) {
    Bits b;
    for (int k = 0; k < 4; k++)
        b.w[k] = low_mask(n - 64 * k);
    return b;
}

// Checks one graph; returns MCS_OK or an error with a message.
mcs_status validate(const mcs_graph &g, const char *which, int idx) {
    char buf[160];
    if (g.n < 0) {
        snprintf(buf, sizeof buf, "%s[%d]: negative vertex count", which, idx);
        return fail(MCS_E_INVALID, buf);
    }
    if (g.n > MCS_MAX_N) {
        snprintf(buf, sizeof buf, "%s[%d]: %d vertices, the limit is %d", which, idx, g.n,
                 MCS_MAX_N);
        return fail(MCS_E_TOO_LARGE, buf);
    }
    if (g.n > 0 && !g.adj) {
        snprintf(buf, sizeof buf, "%s[%d]: adj is NULL", which, idx);
        return fail(MCS_E_INVALID, buf);
    }
    if (g.directed != 0 && g.directed != 1) {
        snprintf(buf, sizeof buf, "%s[%d]: directed must be 0 or 1", which, idx);
        return fail(MCS_E_INVALID, buf);
    }
    const int rw = row_words(g.n);
    for (int i = 0; i < g.n; i++) {
        for (int k = 0; k < rw; k++)
            if (g.adj[(size_t)i * rw + k] & ~low_mask(g.n - 64 * k)) {
                snprintf(buf, sizeof buf, "%s[%d]: row %d has bits at or above n", which, idx, i);
                return fail(MCS_E_INVALID, buf);
            }
        if (in_arc(g, i, i)) {
            snprintf(buf, sizeof buf, "%s[%d]: self loop at vertex %d", which, idx, i);
            return fail(MCS_E_INVALID, buf);
        }
        if (!g.directed)
            for (int j = 0; j < g.n; j++)
                if (in_arc(g, i, j) != in_arc(g, j, i)) {
                    snprintf(buf, sizeof buf, "%s[%d]: undirected graph is not symmetric at (%d,%d)",
                             which, idx, i, j);
                    return fail(MCS_E_INVALID, buf);
                }
    }
    return MCS_OK;
}

// Descending degree (out + in when directed), ties by index (Sec. IV.A).
std::vector<int> degree_order(const mcs_graph &g) {
    std::vector<int> deg(g.n, 0), ord(g.n);
    for (int i = 0; i < g.n; i++)
        for (int j = 0; j < g.n; j++)
            deg[i] += (int)in_arc(g, i, j) + (g.directed ? (int)in_arc(g, j, i) : 0);
    for (int i = 0; i < g.n; i++)
        ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return deg[a] > deg[b]; });
    return ord;
}

// The alternative order of Sec. IV.A ("graph sorting"): weak connected
// components, a component with more non-zero rows per non-zero column first
// (ties: the larger, then the one with the smaller first vertex; components
// without arcs last); within a component, Hellerman-Rarick style, the
// column meeting the most shortest active rows is taken next (ties: the
// smaller index) and leaves the active submatrix; rows whose active length
// reaches zero leave it too; vertices never taken follow in index order.
static bool arc(const mcs_graph &g, int i, int j) { return in_arc(g, i, j); }

std::vector<int> btf_order(const mcs_graph &g) {
    const int n = g.n;
    std::vector<int> comp_of(n, -1);
    std::vector<std::vector<int>> comps;
    for (int s = 0; s < n; s++) {
        if (comp_of[s] >= 0)
            continue;
        std::vector<int> members, todo{s};
        comp_of[s] = (int)comps.size();
        while (!todo.empty()) {
            int u = todo.back();
            todo.pop_back();
            members.push_back(u);
            for (int x = 0; x < n; x++)
                if (comp_of[x] < 0 && (arc(g, u, x) || arc(g, x, u))) {
                    comp_of[x] = comp_of[s];
                    todo.push_back(x);
                }
        }
        std::sort(members.begin(), members.end());
        comps.push_back(members);
    }
    struct Key {
        int no_arcs;
        double neg_ratio;
        int neg_size, first, idx;
    };
    std::vector<Key> keys;
    for (int c = 0; c < (int)comps.size(); c++) {
        const std::vector<int> &m = comps[c];
        int nzr = 0, nzc = 0;
        for (int u : m) {
            bool r = false, col = false;
            for (int x : m) {
                r = r || arc(g, u, x);
                col = col || arc(g, x, u);
            }
            nzr += r;
            nzc += col;
        }
        keys.push_back({nzr == 0 ? 1 : 0, nzr == 0 ? 0.0 : -(double)nzr / nzc,
                        nzr == 0 ? 0 : -(int)m.size(), m[0], c});
    }
    std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) {
        if (a.no_arcs != b.no_arcs)
            return a.no_arcs < b.no_arcs;
        if (a.neg_ratio != b.neg_ratio)
            return a.neg_ratio < b.neg_ratio;
        if (a.neg_size != b.neg_size)
            return a.neg_size < b.neg_size;
        return a.first < b.first;
    });
    std::vector<int> ord;
    for (const Key &k : keys) {
        const std::vector<int> &m = comps[k.idx];
        std::vector<char> row_on(n, 0), col_on(n, 0), taken(n, 0);
        for (int u : m)
            for (int x : m) {
                if (arc(g, u, x)) {
                    row_on[u] = 1;
                    col_on[x] = 1;
                }
            }
        for (;;) {
            int least = n + 1;
            std::vector<int> len(n, 0);
            for (int r : m) {
                if (!row_on[r])
                    continue;
                for (int c : m)
                    len[r] += col_on[c] && arc(g, r, c);
                if (len[r] == 0)
                    row_on[r] = 0;
                else
                    least = std::min(least, len[r]);
            }
            if (least > n)
                break;  // no active row left
            int best = -1, best_hits = -1;
            for (int c : m) {  // ascending: ties go to the smaller index
                if (!col_on[c])
                    continue;
                int hits = 0;
                for (int r : m)
                    hits += row_on[r] && len[r] == least && arc(g, r, c);
                if (hits > best_hits) {
                    best = c;
                    best_hits = hits;
                }
            }
            ord.push_back(best);
            taken[best] = 1;
            col_on[best] = 0;
        }
        for (int u : m)
            if (!taken[u])
                ord.push_back(u);
    }
    return ord;
}

// rows of the relabelled graph: vertex p is original ord[p]
std::vector<Bits> permuted_rows(const mcs_graph &g, const std::vector<int> &ord) {
    std::vector<Bits> rows(g.n);
    for (int p = 0; p < g.n; p++)
        for (int q = 0; q < g.n; q++)
            if (in_arc(g, ord[p], ord[q]))
                rows[p].set(q);
    return rows;
}

std::vector<Bits> transpose_rows(const std::vector<Bits> &rows) {
    int n = (int)rows.size();
    std::vector<Bits> t(n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            if (rows[i].get(j))
                t[j].set(i);
    return t;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

}  // namespace

struct mcs_plan {
    int count = 0;     // search instances on the device
    int pairs = 0;     // the caller's pairs (count, or count / 2 for a portfolio)
    int portfolio = 0; // 1: pair k is instances 2k (degree order) and 2k + 1
                       // (block-triangular order), sharing incumbent word 2k
    int directed = 0;
    int word_bytes = 8;
    int mmax = 0;
    mcs_tuning tun{};
    int64_t node_limit = 0;
    int64_t dead_abs = 0, dead_rel = 0;  // dead-end forecast thresholds (0: off)
    double time_limit_s = 600.0;
    const uint16_t *policy = nullptr;
    int policy_depth = 0, policy_levels = 0, policy_mode = 0;
    int ordering = 0;  // 0: descending degree; 1: components, block-triangular (Sec. IV.A);
                       // 2: both, as a portfolio

    // first device instance of the caller's pair k
    int dev(int k) const { return portfolio ? 2 * k : k; }

    std::vector<mcs::DevInst> inst;
    std::vector<uint8_t> adj;      // packed rows, word_bytes each (4, 8 or 16)
    std::vector<uint8_t> rootcls;  // packed (L, R) pairs
    std::vector<std::vector<int>> ordG, ordH;
    std::vector<int> m;            // min(nG, nH) per instance
    std::vector<int> K0;           // root class count per instance
    std::vector<int> root_bound;   // Eq. 1 at the root per instance
    size_t map_pairs = 0;

    // device layout
    size_t off_inst = 0, off_adj = 0, off_cls = 0, off_inc = 0, off_open = 0, off_nodes = 0,
           off_tbest = 0, off_tproof = 0, off_bestn = 0, off_dead = 0, off_maps = 0, off_glob = 0, off_seq = 0, off_slots = 0,
           off_hstack = 0, hstack_stride = 0,
           ws_bytes = 0;
    int ring_slots = 0, slot_bytes = 0, cap_classes = 0, frames = 0, lds_per_wave = 0;
    int waves_per_block = 4, blocks = 0, waves = 0, lds_per_block = 0;
    int seg_log = 0;   // 3 or 4: searches of 2^seg_log lanes (mcs_seg.hip); 0: one per wavefront
    int seg_bytes = 0, arows = 0;
    double tick_hz = 1e8;

    uint8_t *ws = nullptr;
    bool no_events = false;  // (the static-scratch entry creates no events)
    bool uploaded = false;
    bool launched = false;
    mcs::SearchParams sp{};
    mcs::ResetParams rp{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t gnode_search = nullptr;
    mcs::SearchParams sp_graph{};  // the search parameters the graph's kernel node holds
    // Graph mode stages the inputs and the results in pinned host memory:
    // the graph copies the whole input image in, runs reset + search, and
    // copies the whole result range out, so one replay is a complete solve.
    uint8_t *pin = nullptr;
    size_t pin_in_bytes = 0, pin_out_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = 0.f;

    // results of the last run
    std::vector<int> h_inc, h_open, h_dead;
    std::vector<unsigned long long> h_nodes, h_tbest, h_tproof;
    std::vector<uint16_t> h_maps;
    std::vector<uint8_t> h_out;  // the result range as copied back
    mcs::DevGlobals h_glob{};
    bool have_results = false;

    ~mcs_plan() {
        if (pin)
            (void)hipHostFree(pin);
        if (gexec)
            (void)hipGraphExecDestroy(gexec);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (ev0)
            (void)hipEventDestroy(ev0);
        if (ev1)
            (void)hipEventDestroy(ev1);
    }
};

namespace {

template <typename W>
void put_word(std::vector<uint8_t> &buf, uint64_t x) {
    W w = (W)x;
    const uint8_t *p = (const uint8_t *)&w;
    buf.insert(buf.end(), p, p + sizeof(W));
}

// One row word as the kernels read it: 32, 64, 128 or 256 bits (low
// 64-bit word first).
void pack_word(std::vector<uint8_t> &buf, int word_bytes, const Bits &x) {
    if (word_bytes == 4) {
        put_word<uint32_t>(buf, x.w[0]);
    } else {
        for (int k = 0; k < word_bytes / 8; k++)
            put_word<uint64_t>(buf, x.w[k]);
    }
}

int next_pow2(int x) {
    int p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

}  // namespace

extern "C" {

const char *mcs_status_string(mcs_status s) {
    switch (s) {
    case MCS_OK: return "ok";
    case MCS_LIMIT: return "limit reached (results valid, not all proven optimal)";
    case MCS_E_INVALID: return "invalid input";
    case MCS_E_TOO_LARGE: return "graph too large";
    case MCS_E_DEVICE: return "device error";
    case MCS_E_WORKSPACE: return "workspace missing or too small";
    case MCS_E_INTERNAL: return "internal capacity check failed";
    }
    return "unknown status";
}

const char *mcs_last_error(void) { return g_err.c_str(); }

mcs_status mcs_plan_create(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, mcs_plan **out) {
    g_err.clear();
    if (!out)
        return fail(MCS_E_INVALID, "out is NULL");
    *out = nullptr;
    if (count <= 0)
        return fail(MCS_E_INVALID, "count must be positive");
    if (!G || !H)
        return fail(MCS_E_INVALID, "G or H is NULL");
    // One launch runs one kernel variant: if any pair is directed, all pairs
    // go through the four-way (arc pair) split, which on an undirected graph
    // (in-rows equal to out-rows) gives the same classes as the two-way one.
    int directed = 0;
    for (int i = 0; i < count; i++) {
        mcs_status s = validate(G[i], "G", i);
        if (s != MCS_OK)
            return s;
        s = validate(H[i], "H", i);
        if (s != MCS_OK)
            return s;
        if (G[i].directed != H[i].directed)
            return fail(MCS_E_INVALID, "G and H of a pair differ in directedness");
        if ((G[i].label == nullptr) != (H[i].label == nullptr))
            return fail(MCS_E_INVALID, "G and H of a pair differ in having labels");
        directed |= G[i].directed;
    }

    mcs_plan *p = new mcs_plan();
    p->pairs = count;
    p->count = count;
    p->directed = directed;
    if (opts) {
        if (opts->tuning)
            p->tun = *opts->tuning;
        if (opts->policy) {
            if (opts->policy_depth < 0 || opts->policy_depth > 8) {
                delete p;
                return fail(MCS_E_INVALID, "policy_depth must be in 0..8");
            }
            if ((uintptr_t)opts->policy % 16 != 0) {
                delete p;
                return fail(MCS_E_INVALID, "policy parameters must be 16-byte aligned");
            }
            p->policy = opts->policy;
            p->policy_depth = opts->policy_depth;
            p->policy_mode = opts->policy_mode ? (opts->policy_mode & 3) : 2;
            p->policy_levels = opts->policy_depth + 1;
        }
        p->node_limit = opts->node_limit > 0 ? opts->node_limit : 0;
        if (opts->deadend_nodes < 0 || opts->deadend_ratio < 0) {
            delete p;
            return fail(MCS_E_INVALID, "deadend_nodes and deadend_ratio must be >= 0");
        }
        p->dead_abs = opts->deadend_nodes;
        p->dead_rel = opts->deadend_ratio;
        if (opts->ordering < 0 || opts->ordering > 2) {
            delete p;
            return fail(MCS_E_INVALID, "ordering must be 0 (degree), 1 (block-triangular) or "
                                       "2 (both, as a portfolio)");
        }
        p->ordering = opts->ordering;
        if (p->ordering == 2) {
            p->portfolio = 1;
            p->count = 2 * count;
        }
        if (opts->time_limit_s > 0)
            p->time_limit_s = opts->time_limit_s;
    }
    int nmax = 0;
    for (int i = 0; i < count; i++)
        nmax = std::max(nmax, std::max(G[i].n, H[i].n));
    p->word_bytes = nmax <= 32 ? 4 : nmax <= 64 ? 8 : nmax <= 128 ? 16 : 32;
    if (p->policy && p->word_bytes > 8) {
        delete p;
        return fail(MCS_E_INVALID, "the learned policy takes graphs of at most 64 vertices");
    }
    const int NB = 8 * p->word_bytes;
    const int R = directed ? 4 : 2;

    const int ndev = p->count;
    p->inst.resize(ndev);
    p->ordG.resize(ndev);
    p->ordH.resize(ndev);
    p->m.resize(ndev);
    uint32_t cls_off = 0;
    size_t map_off = 0;
    for (int i = 0; i < ndev; i++) {
        const int k = p->portfolio ? i >> 1 : i;
        const mcs_graph &g = G[k], &h = H[k];
        const int order = p->portfolio ? (i & 1) : p->ordering;
        p->ordG[i] = order == 1 ? btf_order(g) : degree_order(g);
        p->ordH[i] = order == 1 ? btf_order(h) : degree_order(h);
        std::vector<Bits> rg = permuted_rows(g, p->ordG[i]);
        std::vector<Bits> rh = permuted_rows(h, p->ordH[i]);
        std::vector<std::vector<Bits>> sets = {rg, rh};
        if (directed) {
            sets.push_back(transpose_rows(rg));
            sets.push_back(transpose_rows(rh));
        }
        for (int s = 0; s < R; s++)
            for (int j = 0; j < NB; j++)
                pack_word(p->adj, p->word_bytes, j < (int)sets[s].size() ? sets[s][j] : Bits{});

        // root classes
        int K0 = 0;
        if (g.n > 0 && h.n > 0) {
            if (!g.label) {
                pack_word(p->rootcls, p->word_bytes, first_n(g.n));
                pack_word(p->rootcls, p->word_bytes, first_n(h.n));
                K0 = 1;
            } else {
                std::vector<int> seen;
                for (int a = 0; a < g.n; a++) {
                    int lab = g.label[p->ordG[i][a]];
                    if (std::find(seen.begin(), seen.end(), lab) != seen.end())
                        continue;
                    seen.push_back(lab);
                    Bits L, Rm;
                    for (int b = 0; b < g.n; b++)
                        if (g.label[p->ordG[i][b]] == lab)
                            L.set(b);
                    for (int b = 0; b < h.n; b++)
                        if (h.label[p->ordH[i][b]] == lab)
                            Rm.set(b);
                    if (!Rm.any())
                        continue;
                    pack_word(p->rootcls, p->word_bytes, L);
                    pack_word(p->rootcls, p->word_bytes, Rm);
                    K0++;
                }
            }
        }
        int mi = std::min(g.n, h.n);
        p->m[i] = mi;
        p->mmax = std::max(p->mmax, mi);
        mcs::DevInst di{};
        di.nG = (uint8_t)g.n;
        di.nH = (uint8_t)h.n;
        di.K0 = (uint8_t)K0;
        di.cls_off = cls_off;
        di.map_off = (uint32_t)map_off;
        di.lb = 0;
        di.target = 0;
        di.inc_slot = p->portfolio ? (i & ~1) : i;
        di.twin = p->portfolio ? (i ^ 1) : -1;
        di.dead_on = p->dead_abs > 0 ? 1 : 0;
        p->inst[i] = di;
        p->K0.push_back(K0);
        // Eq. 1 at the root: the largest size any goal needs to consider
        int rb = 0;
        if (g.n > 0 && h.n > 0) {
            if (!g.label) {
                rb = std::min(g.n, h.n);
            } else {
                std::vector<int> seen;
                for (int a = 0; a < g.n; a++) {
                    int lab = g.label[a];
                    if (std::find(seen.begin(), seen.end(), lab) != seen.end())
                        continue;
                    seen.push_back(lab);
                    int cg = 0, ch = 0;
                    for (int b = 0; b < g.n; b++)
                        cg += g.label[b] == lab;
                    for (int b = 0; b < h.n; b++)
                        ch += h.label[b] == lab;
                    rb += std::min(cg, ch);
                }
            }
        }
        p->root_bound.push_back(rb);
        cls_off += (uint32_t)K0;
        map_off += (size_t)mi * (mi + 1) / 2;
    }
    if (p->rootcls.empty())
        pack_word(p->rootcls, p->word_bytes, Bits{}), pack_word(p->rootcls, p->word_bytes, Bits{});
    p->map_pairs = std::max<size_t>(map_off, 1);
    // The worst case of the depth-first class stack: frame t holds at most
    // m - t classes.
    const int full_cap = std::max(1, p->mmax * (p->mmax + 1) / 2);
    // The LDS part must hold any one frame at its start (a root's classes, a
    // taken record's), so never fewer than m classes.
    const int min_cap = std::min(full_cap, std::max(1, p->mmax));
    p->frames = p->mmax + 1;

    // launch shape
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        dev = 0;
    int cus = 256, max_lds_block = 65536, lds_cu = 163840, clock_khz = 100000;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&max_lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (lds_cu < max_lds_block)
        lds_cu = max_lds_block;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        clock_khz <= 0)
        clock_khz = 100000;
    (void)hipGetLastError();
    p->tick_hz = (double)clock_khz * 1000.0;
    const bool wide = p->word_bytes >= 16;
    // Search layout: one search per lane segment of 16 (or 8) lanes
    // (mcs_seg.hip), or one per wavefront (mcs_search.hip: needed for
    // 128-bit rows and for the learned policy, which scores one vertex per
    // lane).
    {
        const int sl = p->tun.seg_lanes;
        if (sl != 0 && sl != 4 && sl != 8 && sl != 16 && sl != 64) {
            delete p;
            return fail(MCS_E_INVALID, "seg_lanes must be 0, 4, 8, 16 or 64");
        }
        if (wide || p->policy || sl == 64)
            p->seg_log = 0;
        else
            p->seg_log = sl == 4 ? 2 : sl == 16 ? 4 : 3;  // default: 8 lanes
    }
    const int nseg = p->seg_log ? 64 >> p->seg_log : 1;
    if (p->seg_log) {
        // adjacency rows a segment keeps: the batch's largest graph, to 4
        int nmax_all = 0;
        for (int i = 0; i < count; i++)
            nmax_all = std::max(nmax_all, std::max(G[i].n, H[i].n));
        p->arows = std::min(NB, std::max(4, (nmax_all + 3) & ~3));
    }
    auto per_wave = [&](int cap) {
        if (p->seg_log)
            return nseg * mcs::seg_layout(p->word_bytes, directed, cap, p->arows, p->frames).total;
        return mcs::lds_layout(p->word_bytes, directed, wide ? -1 : cap, p->frames,
                               p->policy_levels).total;
    };
    // LDS bytes one wavefront may use when wpc of them share a CU
    // (workgroups of 4; each workgroup's LDS is its wavefronts' parts plus
    // the kernel's static 256 bytes, allocated in granules), and the class
    // stack's LDS part that leaves to each segmented search.
    auto wave_share = [&](int wpc) {
        const int blocks_cu = std::max(1, (wpc + 3) / 4);
        return ((lds_cu / blocks_cu) / kLdsGranule * kLdsGranule - 256) / 4;
    };
    auto seg_cap_at = [&](int wpc) {
        const int room = wave_share(wpc) / nseg - per_wave(0) / nseg - 16;
        return std::max(0, std::min(full_cap, room / (2 * p->word_bytes)));
    };
    // Default wavefronts: about 96 searches per instance, between 8 and 24
    // per CU, for one search per wavefront (4 and 16 with 128-bit rows, whose
    // larger state fits fewer), so one hard instance alone still splits
    // across thousands of searches.  The segmented kernel takes about 256
    // searches per instance, at least 8 wavefronts per CU and at most 16, 12
    // or 8 (its registers allow 4 per SIMD): the most whose LDS still leaves
    // each search an LDS part of about 32 classes.  One search is a long
    // dependent chain of steps, so several wavefronts per SIMD fill the VALU
    // issue slots while there is work for them; past what the instances can
    // keep busy, more searches only split the work into ever smaller
    // donations (measured: 60 pairs G(30, p) take 439 ms at 8 wavefronts per
    // CU, 465 ms at 16 and 795 ms at 2.8; the 4,096 batched pairs 23.5 s at
    // 16 and 27-28 s at 12).
    int seg_wpc = 8;
    if (p->seg_log) {
        const int want_cap = std::min(full_cap, std::max(min_cap, 32));
        for (int wpc : {16, 12}) {
            if (seg_cap_at(wpc) >= want_cap) {
                seg_wpc = wpc;
                break;
            }
        }
    }
    const int want_waves =
        p->tun.waves_per_cu > 0 ? p->tun.waves_per_cu * cus
        : p->seg_log ? std::min(seg_wpc * cus, std::max(8 * cus, (256 * ndev + nseg - 1) / nseg))
        : wide       ? std::max(4 * cus, std::min(16 * cus, 96 * ndev))
                     : std::max(8 * cus, std::min(24 * cus, 96 * ndev));
    const int target_wpc = p->tun.single_wave ? 1 : std::max(1, (want_waves + cus - 1) / cus);
    if (!p->seg_log) {
        // One search per wavefront: the whole worst case, in LDS (at most
        // 2081 classes of 16 bytes for 64 vertices) or, with 128-bit rows,
        // in the wavefront's slice of HBM (up to 264 KB), so a child always
        // has room on its stack.
        p->cap_classes = full_cap;
    } else if (p->tun.stack_classes > 0) {
        p->cap_classes = std::max(min_cap, std::min(full_cap, p->tun.stack_classes));
    } else {
        // Segments: the whole worst case in LDS if target_wpc wavefronts
        // still fit in a CU, else the largest LDS part that lets them; the
        // rest of each search's worst case is in HBM.
        p->cap_classes = full_cap;
        if (per_wave(full_cap) > wave_share(target_wpc))
            p->cap_classes = std::max(min_cap, seg_cap_at(target_wpc));
    }
    max_lds_block -= 256;  // the kernel's static LDS (its parameter copy)
    if (p->seg_log && per_wave(p->cap_classes) > max_lds_block) {
        // one wavefront's stacks must fit in one workgroup's LDS
        const int room = max_lds_block / nseg - per_wave(0) / nseg - 16;
        p->cap_classes = std::max(min_cap, std::min(p->cap_classes, room / (2 * p->word_bytes)));
    }
    p->lds_per_wave = per_wave(p->cap_classes);
    if (p->seg_log)
        p->seg_bytes = p->lds_per_wave / nseg;
    int wpb = 4;
    while (wpb > 1 && wpb * p->lds_per_wave > max_lds_block)
        wpb >>= 1;
    if (p->lds_per_wave > max_lds_block) {
        delete p;
        return fail(MCS_E_INTERNAL, "LDS of one wavefront exceeds the workgroup limit");
    }
    p->waves_per_block = wpb;
    p->lds_per_block = wpb * p->lds_per_wave;
    const void *kern = p->seg_log ? mcs_internal_seg_kernel(p->word_bytes, directed, p->seg_log)
                                  : mcs_internal_search_kernel(p->word_bytes, directed,
                                                               p->policy != nullptr);
    int per_cu = 0;
    if (p->lds_per_block > 65536)
        (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  p->lds_per_block);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb,
                                                     (size_t)p->lds_per_block) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    {
        // Never more workgroups than stay resident together: a persistent
        // grid's extra workgroups would only start once the first ones end.
        // LDS is counted in whole granules here, on top of the occupancy
        // query.
        const int blk = (p->lds_per_block + 256 + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
        per_cu = std::max(1, std::min(per_cu, lds_cu / blk));
    }
    p->blocks = per_cu * cus;
    if (p->tun.single_wave)
        p->blocks = 1;
    else
        p->blocks = std::max(1, std::min(p->blocks, (want_waves + wpb - 1) / wpb));
    p->waves = p->blocks * wpb;

    {
        int total = p->tun.ring_slots > 0 ? p->tun.ring_slots : std::max(1024, 2 * p->waves);
        p->ring_slots = next_pow2(std::max(2, (total + mcs::kRings - 1) / mcs::kRings));
    }
    p->slot_bytes = mcs::slot_bytes_for(p->word_bytes, p->mmax);
    // HBM class stacks: a wavefront's whole stack with 128-bit rows; with
    // segments, the part of each search's worst case above its LDS part
    // (frames placed there start at cap_classes and total at most full_cap
    // classes)
    size_t hstacks = 0;
    if (wide) {
        p->hstack_stride = (long long)align256((size_t)(p->cap_classes + 1) * 2 * p->word_bytes);
        hstacks = (size_t)p->waves;
    } else if (p->seg_log && p->cap_classes < full_cap) {
        p->hstack_stride = (long long)align256((size_t)full_cap * 2 * p->word_bytes);
        hstacks = (size_t)p->waves * (size_t)nseg;
    }
    if (p->seg_log &&
        (long long)p->cap_classes + p->hstack_stride / (2 * p->word_bytes) > 4095) {
        // a segment's frame header keeps a frame's first class in 12 bits
        delete p;
        return fail(MCS_E_INTERNAL, "class stack indices exceed the frame header's 12 bits");
    }

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p->off_inst = take(sizeof(mcs::DevInst) * ndev);
    p->off_adj = take(p->adj.size());
    p->off_cls = take(p->rootcls.size());
    p->off_inc = take(sizeof(int) * ndev);
    p->off_open = take(sizeof(int) * ndev);
    p->off_nodes = take(sizeof(unsigned long long) * ndev);
    p->off_tbest = take(sizeof(unsigned long long) * ndev);
    p->off_tproof = take(sizeof(unsigned long long) * ndev);
    p->off_bestn = take(sizeof(unsigned long long) * ndev);
    p->off_dead = take(sizeof(int) * ndev);
    p->off_maps = take(sizeof(uint16_t) * p->map_pairs);
    p->off_glob = take(sizeof(mcs::DevGlobals));
    p->off_seq = take(sizeof(unsigned long long) * mcs::kRings * p->ring_slots);
    p->off_slots = take((size_t)p->slot_bytes * mcs::kRings * p->ring_slots);
    p->off_hstack = take((size_t)p->hstack_stride * hstacks);
    p->ws_bytes = o;
    *out = p;
    return MCS_OK;
}

size_t mcs_plan_workspace_size(const mcs_plan *p) { return p ? p->ws_bytes : 0; }

mcs_status mcs_plan_upload(mcs_plan *p, void *workspace, size_t bytes, void *stream) {
    g_err.clear();
    if (!p)
        return fail(MCS_E_INVALID, "plan is NULL");
    if (!workspace || bytes < p->ws_bytes || ((uintptr_t)workspace & 255))
        return fail(MCS_E_WORKSPACE, "workspace must be at least mcs_plan_workspace_size bytes, "
                                     "256-byte aligned");
    if (p->ws != (uint8_t *)workspace && p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
        p->gnode_search = nullptr;
    }
    p->ws = (uint8_t *)workspace;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_inst, p->inst.data(), sizeof(mcs::DevInst) * p->count,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_adj, p->adj.data(), p->adj.size(), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_cls, p->rootcls.data(), p->rootcls.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));

    mcs::SearchParams &sp = p->sp;
    sp = mcs::SearchParams{};
    sp.inst = (const mcs::DevInst *)(p->ws + p->off_inst);
    sp.adj = p->ws + p->off_adj;
    sp.rootcls = p->ws + p->off_cls;
    sp.inc = (int *)(p->ws + p->off_inc);
    sp.open = (int *)(p->ws + p->off_open);
    sp.nodes = (unsigned long long *)(p->ws + p->off_nodes);
    sp.t_best = (unsigned long long *)(p->ws + p->off_tbest);
    sp.t_proof = (unsigned long long *)(p->ws + p->off_tproof);
    sp.best_nodes = (unsigned long long *)(p->ws + p->off_bestn);
    sp.dead = (int *)(p->ws + p->off_dead);
    sp.maps = (uint16_t *)(p->ws + p->off_maps);
    sp.g = (mcs::DevGlobals *)(p->ws + p->off_glob);
    sp.seq = (unsigned long long *)(p->ws + p->off_seq);
    sp.slots = p->ws + p->off_slots;
    sp.count = p->count;
    sp.ring_slots = p->ring_slots;
    sp.slot_bytes = p->slot_bytes;
    sp.cap_classes = p->cap_classes;
    sp.frames = p->frames;
    sp.lds_per_wave = p->lds_per_wave;
    int cm = p->tun.children_per_wave;
    sp.cmax = (cm == 1 || cm == 2 || cm == 4 || cm == 8) ? cm : 8;
    sp.donate_low = p->tun.donate_low > 0 ? p->tun.donate_low
                                          : (p->tun.donate_low < 0 ? -1 : 2);
    // Any frame may be handed out by default: a depth cut-off left the last
    // hard instance's deep subtrees to one search while the rest idled
    // (measured on the batched workload: 27-28 s instead of 30-37 s).
    sp.donate_depth = p->tun.donate_depth > 0 ? p->tun.donate_depth : std::max(1, p->mmax);
    // (at most 2^16: the kernel's per-check step counters are 32-bit)
    sp.check_interval = p->tun.check_interval > 0 ? std::min(p->tun.check_interval, 65536) : 128;
    sp.reprune = p->tun.no_reprune ? 0 : 1;
    sp.backoff_max = p->tun.backoff_max > 0 ? std::min(p->tun.backoff_max, 1024) : 32;
    sp.single_wave = p->tun.single_wave ? 1 : 0;
    sp.policy = p->policy;
    sp.policy_depth = p->policy_depth;
    sp.policy_levels = p->policy_levels;
    sp.policy_mode = p->policy_mode;
    double ticks = p->time_limit_s * p->tick_hz;
    sp.limit_ticks = ticks > 9e18 ? (unsigned long long)9e18 : (unsigned long long)ticks;
    sp.node_limit = p->node_limit;
    sp.dead_abs = p->dead_abs;
    sp.dead_rel = p->dead_rel;
    sp.hstack = p->hstack_stride ? p->ws + p->off_hstack : nullptr;
    sp.hstack_stride = p->hstack_stride;
    sp.seg_log = p->seg_log;
    sp.seg_bytes = p->seg_bytes;
    sp.arows = p->arows;

    mcs::ResetParams &rp = p->rp;
    rp.inst = sp.inst;
    rp.inc = sp.inc;
    rp.open = sp.open;
    rp.nodes = sp.nodes;
    rp.t_best = sp.t_best;
    rp.t_proof = sp.t_proof;
    rp.best_nodes = sp.best_nodes;
    rp.dead = sp.dead;
    rp.g = sp.g;
    rp.seq = sp.seq;
    rp.count = p->count;
    rp.ring_slots = p->ring_slots;
    p->uploaded = true;
    return MCS_OK;
}

static void *search_fn(const mcs_plan *p) {
    return p->seg_log ? mcs_internal_seg_kernel(p->word_bytes, p->directed, p->seg_log)
                      : mcs_internal_search_kernel(p->word_bytes, p->directed, p->policy != nullptr);
}

static mcs_status launch_direct(mcs_plan *p, hipStream_t s) {
    const void *kr = mcs_internal_reset_kernel();
    const void *ks = search_fn(p);
    int n = std::max(p->count, mcs::kRings * p->ring_slots);
    int rb = std::min(1024, (n + 255) / 256);
    void *ra[] = {&p->rp};
    HIP_TRY(hipLaunchKernel(kr, dim3(rb), dim3(256), ra, 0, s));
    if (p->ev0)
        HIP_TRY(hipEventRecord(p->ev0, s));
    void *sa[] = {&p->sp};
    HIP_TRY(hipLaunchKernel(ks, dim3(p->blocks), dim3(64 * p->waves_per_block), sa,
                            (size_t)p->lds_per_block, s));
    if (p->ev1)
        HIP_TRY(hipEventRecord(p->ev1, s));
    return MCS_OK;
}

// The input image (descriptors, rows, root classes) and the result range
// (incumbents through the globals) are each one contiguous part of the
// workspace, so a graph moves each with a single copy.
static size_t in_begin(const mcs_plan *p) { return p->off_inst; }
static size_t in_end(const mcs_plan *p) { return p->off_cls + p->rootcls.size(); }
static size_t out_begin(const mcs_plan *p) { return p->off_inc; }
static size_t out_end(const mcs_plan *p) { return p->off_glob + sizeof(mcs::DevGlobals); }

static void stage_inputs(mcs_plan *p) {
    uint8_t *img = p->pin;
    const size_t b = in_begin(p);
    std::memset(img, 0, p->pin_in_bytes);
    std::memcpy(img + (p->off_inst - b), p->inst.data(), sizeof(mcs::DevInst) * p->count);
    std::memcpy(img + (p->off_adj - b), p->adj.data(), p->adj.size());
    std::memcpy(img + (p->off_cls - b), p->rootcls.data(), p->rootcls.size());
}

// HIP graph of one complete solve: input copy, reset kernel, search kernel
// (bracketed by the timing events), result copy.  No memset nodes: the reset
// kernel clears the state with plain stores.
static mcs_status build_graph(mcs_plan *p) {
    if (!p->pin) {
        p->pin_in_bytes = in_end(p) - in_begin(p);
        p->pin_out_bytes = out_end(p) - out_begin(p);
        HIP_TRY(hipHostMalloc((void **)&p->pin, p->pin_in_bytes + p->pin_out_bytes,
                              hipHostMallocDefault));
    }
    stage_inputs(p);
    HIP_TRY(hipGraphCreate(&p->graph, 0));
    hipGraphNode_t nin = nullptr, nr = nullptr, ne0 = nullptr, ns = nullptr, ne1 = nullptr,
                   nout = nullptr;
    HIP_TRY(hipGraphAddMemcpyNode1D(&nin, p->graph, nullptr, 0, p->ws + in_begin(p), p->pin,
                                    p->pin_in_bytes, hipMemcpyHostToDevice));
    int n = std::max(p->count, mcs::kRings * p->ring_slots);
    void *ra[] = {&p->rp};
    void *sa[] = {&p->sp};
    hipKernelNodeParams kp{};
    kp.func = mcs_internal_reset_kernel();
    kp.gridDim = dim3(std::min(1024, (n + 255) / 256));
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = ra;
    kp.extra = nullptr;
    HIP_TRY(hipGraphAddKernelNode(&nr, p->graph, &nin, 1, &kp));
    HIP_TRY(hipGraphAddEventRecordNode(&ne0, p->graph, &nr, 1, p->ev0));
    hipKernelNodeParams ks{};
    ks.func = search_fn(p);
    ks.gridDim = dim3(p->blocks);
    ks.blockDim = dim3(64 * p->waves_per_block);
    ks.sharedMemBytes = (unsigned)p->lds_per_block;
    ks.kernelParams = sa;
    ks.extra = nullptr;
    HIP_TRY(hipGraphAddKernelNode(&ns, p->graph, &ne0, 1, &ks));
    HIP_TRY(hipGraphAddEventRecordNode(&ne1, p->graph, &ns, 1, p->ev1));
    HIP_TRY(hipGraphAddMemcpyNode1D(&nout, p->graph, &ne1, 1, p->pin + p->pin_in_bytes,
                                    p->ws + out_begin(p), p->pin_out_bytes,
                                    hipMemcpyDeviceToHost));
    HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    p->gnode_search = ns;
    p->sp_graph = p->sp;
    return MCS_OK;
}

// Kernel-node arguments are copied when the node is made: a run after the
// search parameters changed (a goal run dropping the node limit, say) must
// hand the new ones to the instantiated graph.
static mcs_status refresh_graph_params(mcs_plan *p) {
    if (std::memcmp(&p->sp_graph, &p->sp, sizeof(p->sp)) == 0)
        return MCS_OK;
    void *sa[] = {&p->sp};
    hipKernelNodeParams ks{};
    ks.func = search_fn(p);
    ks.gridDim = dim3(p->blocks);
    ks.blockDim = dim3(64 * p->waves_per_block);
    ks.sharedMemBytes = (unsigned)p->lds_per_block;
    ks.kernelParams = sa;
    ks.extra = nullptr;
    HIP_TRY(hipGraphExecKernelNodeSetParams(p->gexec, p->gnode_search, &ks));
    p->sp_graph = p->sp;
    return MCS_OK;
}

mcs_status mcs_plan_run(mcs_plan *p, void *stream) {
    g_err.clear();
    if (!p)
        return fail(MCS_E_INVALID, "plan is NULL");
    if (!p->uploaded)
        return fail(MCS_E_WORKSPACE, "mcs_plan_upload has not been called");
    hipStream_t s = as_stream(stream);
    if (!p->ev0 && !p->no_events) {
        HIP_TRY(hipEventCreate(&p->ev0));
        HIP_TRY(hipEventCreate(&p->ev1));
    }
    p->have_results = false;
    p->launched = false;
    if (p->tun.use_graph) {
        if (!p->gexec) {
            mcs_status st = build_graph(p);
            if (st != MCS_OK)
                return st;
        } else {
            mcs_status st = refresh_graph_params(p);
            if (st != MCS_OK)
                return st;
        }
        HIP_TRY(hipGraphLaunch(p->gexec, s));
    } else {
        mcs_status st = launch_direct(p, s);
        if (st != MCS_OK)
            return st;
    }
    p->launched = true;
    return MCS_OK;
}

mcs_status mcs_plan_results(mcs_plan *p, mcs_result *res, void *stream) {
    g_err.clear();
    if (!p)
        return fail(MCS_E_INVALID, "plan is NULL");
    if (!p->launched)
        return fail(MCS_E_INVALID, "mcs_plan_run has not been called");
    hipStream_t s = as_stream(stream);
    int n = p->count;
    const size_t ob = out_begin(p);
    p->h_out.resize(out_end(p) - ob);
    if (p->tun.use_graph && p->gexec) {
        // the graph's last node already copied the result range to pinned memory
        HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(p->h_out.data(), p->pin + p->pin_in_bytes, p->h_out.size());
    } else {
        HIP_TRY(hipMemcpyAsync(p->h_out.data(), p->ws + ob, p->h_out.size(),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    HIP_TRY(hipGetLastError());
    const uint8_t *o = p->h_out.data();
    p->h_inc.assign((const int *)(o + (p->off_inc - ob)), (const int *)(o + (p->off_inc - ob)) + n);
    p->h_open.assign((const int *)(o + (p->off_open - ob)),
                     (const int *)(o + (p->off_open - ob)) + n);
    p->h_dead.assign((const int *)(o + (p->off_dead - ob)),
                     (const int *)(o + (p->off_dead - ob)) + n);
    auto u64s = [&](size_t off) {
        const unsigned long long *q = (const unsigned long long *)(o + (off - ob));
        return std::vector<unsigned long long>(q, q + n);
    };
    p->h_nodes = u64s(p->off_nodes);
    p->h_tbest = u64s(p->off_tbest);
    p->h_tproof = u64s(p->off_tproof);
    p->h_maps.assign((const uint16_t *)(o + (p->off_maps - ob)),
                     (const uint16_t *)(o + (p->off_maps - ob)) + p->map_pairs);
    std::memcpy(&p->h_glob, o + (p->off_glob - ob), sizeof(mcs::DevGlobals));
    if (p->ev0 && hipEventElapsedTime(&p->last_ms, p->ev0, p->ev1) != hipSuccess) {
        (void)hipGetLastError();
        p->last_ms = 0.f;
    }
    p->have_results = true;
    if (p->h_glob.error)
        return fail(MCS_E_INTERNAL,
                    p->h_glob.error == 2   ? "a search produced a mapping larger than the smaller graph"
                    : p->h_glob.error == 3 ? "a search's class stack grew past its worst case"
                                           : "a search wavefront hit an internal capacity check");

    const unsigned long long mask48 = 0xFFFFFFFFFFFFull;
    const unsigned long long t0 = p->h_glob.t0;
    bool all_proven = true;
    for (int k = 0; k < p->pairs; k++) {
        mcs_result &r = res[k];
        const int i0 = p->dev(k), i1 = p->portfolio ? i0 + 1 : i0;
        const int size = p->h_inc[p->inst[i0].inc_slot];
        // a pair is proven once either of its searches finished (a portfolio
        // twin that saw its partner finish ends at once, proving nothing new)
        bool proven = false;
        unsigned long long tp = ~0ull;
        int64_t nodes = 0;
        for (int i = i0; i <= i1; i++) {
            if (p->h_tproof[i] != 0 && p->h_open[i] == 0 && !p->h_dead[i]) {
                proven = true;
                tp = std::min(tp, p->h_tproof[i]);
            }
            nodes += (int64_t)p->h_nodes[i];
        }
        all_proven = all_proven && proven;
        r.size = size;
        r.optimal = proven ? 1 : 0;
        r.nodes = nodes;
        r.t_proof_s = proven ? (double)(tp - t0) / p->tick_hz : 0.0;
        r.t_best_s = 0.0;
        // the mapping of the final size sits in the slots of the search that
        // raised the incumbent to it (exactly one twin of a portfolio pair)
        for (int i = i0; i <= i1; i++) {
            const unsigned long long kb = p->h_tbest[i];
            if (!(size > p->inst[i].lb && size > 0 && (int)(kb >> 48) == size))
                continue;
            r.t_best_s = (double)(((kb & mask48) - (t0 & mask48)) & mask48) / p->tick_hz;
            size_t off = p->inst[i].map_off + (size_t)size * (size - 1) / 2;
            for (int j = 0; j < size; j++) {
                uint16_t e = p->h_maps[off + j];
                int pg = e & 0xFF, ph = e >> 8;
                if (r.map_g)
                    r.map_g[j] = p->ordG[i][pg];
                if (r.map_h)
                    r.map_h[j] = p->ordH[i][ph];
            }
            break;
        }
    }
    return all_proven ? MCS_OK : MCS_LIMIT;
}

mcs_status mcs_plan_stats(const mcs_plan *p, mcs_stats *st) {
    if (!p || !st)
        return fail(MCS_E_INVALID, "NULL argument");
    if (!p->have_results)
        return fail(MCS_E_INVALID, "no results yet");
    mcs_stats z{};
    for (int i = 0; i < p->count; i++)
        z.nodes += (int64_t)p->h_nodes[i];
    z.batches = (int64_t)p->h_glob.batches;
    z.children = (int64_t)p->h_glob.children;
    z.lane_slots = (int64_t)p->h_glob.lane_slots;
    z.donations = (int64_t)p->h_glob.donations;
    z.pops = (int64_t)p->h_glob.pops;
    z.waves = p->waves;
    z.blocks = p->blocks;
    z.lds_per_wave = p->lds_per_wave;
    z.stopped = p->h_glob.stop ? 1 : 0;
    z.kernel_ms = p->last_ms;
    z.busy_wave_s = (double)p->h_glob.busy_ticks / p->tick_hz;
    z.hbm_frames = (int64_t)p->h_glob.hbm_frames;
    z.sleep_wave_s = (double)p->h_glob.sleep_ticks / p->tick_hz;
    // Algorithmic LDS bytes: each child batch reads the rows of v and of
    // its C partners (one word each, two when directed); each pushed frame's
    // classes (L and R words) are written once and read twice (at the descent
    // and when the search returns to the frame).
    {
        // (the segmented kernel reads both rows per child; "batches" are its steps)
        const int64_t rows = p->seg_log ? 2 * (int64_t)p->h_glob.children
                                        : (int64_t)p->h_glob.batches + (int64_t)p->h_glob.children;
        const int rw = (p->directed ? 2 : 1) * p->word_bytes;
        z.lds_bytes = rows * rw + (int64_t)p->h_glob.pushed_classes * 3 * 2 * p->word_bytes;
    }
    z.node_classes = (int64_t)p->h_glob.node_classes;
    z.stack_classes = p->cap_classes;
    z.max_stack_used = p->h_glob.max_stack;
    *st = z;
    return MCS_OK;
}

// Per pair: the incumbent the next run starts from (lb), the size at which
// it stops (target, 0: none), whether the dead-end forecast may give it up,
// and whether it is skipped; copied into the device descriptors.
static mcs_status apply_bounds(mcs_plan *p, const int32_t *lb, const int32_t *target,
                               const int32_t *dead_on, const int32_t *skip, void *stream) {
    for (int i = 0; i < p->count; i++) {
        const int k = p->portfolio ? i >> 1 : i;
        mcs::DevInst &di = p->inst[i];
        di.K0 = (uint8_t)(skip[k] ? 0 : p->K0[i]);
        di.lb = lb[k];
        di.target = target[k];
        di.dead_on = dead_on[k];
    }
    if (p->pin)
        stage_inputs(p);  // a graph replay copies the descriptors in from here
    HIP_TRY(hipMemcpyAsync(p->ws + p->off_inst, p->inst.data(), sizeof(mcs::DevInst) * p->count,
                           hipMemcpyHostToDevice, as_stream(stream)));
    HIP_TRY(hipStreamSynchronize(as_stream(stream)));
    return MCS_OK;
}

mcs_status mcs_plan_set_goals(mcs_plan *p, const int32_t *goal, void *stream) {
    g_err.clear();
    if (!p || !goal)
        return fail(MCS_E_INVALID, "NULL argument");
    if (!p->uploaded)
        return fail(MCS_E_WORKSPACE, "mcs_plan_upload has not been called");
    const int n = p->pairs;
    std::vector<int32_t> lb(n), target(n), don(n), skip(n);
    for (int k = 0; k < n; k++) {
        if (goal[k] > p->m[p->dev(k)])
            return fail(MCS_E_INVALID, "a goal exceeds min(nG, nH)");
        lb[k] = goal[k] > 0 ? goal[k] - 1 : 0;
        target[k] = goal[k] > 0 ? goal[k] : 0;
        don[k] = goal[k] == 0 && p->dead_abs > 0 ? 1 : 0;
        skip[k] = goal[k] < 0 ? 1 : 0;
    }
    return apply_bounds(p, lb.data(), target.data(), don.data(), skip.data(), stream);
}

mcs_status mcs_plan_root_bounds(const mcs_plan *p, int32_t *bounds) {
    if (!p || !bounds)
        return fail(MCS_E_INVALID, "NULL argument");
    for (int k = 0; k < p->pairs; k++)
        bounds[k] = p->root_bound[p->dev(k)];
    return MCS_OK;
}

void mcs_plan_destroy(mcs_plan *p) { delete p; }

// Goal-directed search over a batch (paper Sec. IV.A).  Every pair keeps a
// lower bound lo (the best mapping found, kept) and an upper bound hi (Eq. 1
// at the root, lowered by every refuted goal); it is settled once lo == hi.
// Each launch runs every unsettled pair in one of two kinds of run:
//   goal run g: incumbent g - 1, stop at the first mapping of size >= g;
//     a mapping raises lo, a finished search without one sets hi = g - 1;
//   plain run from s: incumbent s, no stop, the dead-end forecast on (for
//     the dead-end strategies); a finished search settles the pair (its best
//     mapping if it found one above s, else hi = s).
// strategy 0 (top-down): goal runs at hi, hi - 1, ...: the first goal
//   reached is the optimum.
// strategy 1 (bound correction by bisection): a plain run bounded by
//   opts->node_limit gives lo (and may finish); then goal runs at the middle
//   of (lo, hi].
// strategies 2 and 3 (dead-end bound correction): plain runs with the
//   dead-end forecast; a pair forecast to be in a dead end (too many nodes
//   since its incumbent last rose) restarts from s = max(lo, s) + step -- the
//   bound raised by 1 (strategy 2) or by a step that doubles at each
//   forecast, 1, 2, 4, ... (strategy 3) -- so only mappings above s are
//   looked for; a raised bound found unreachable (a finished run with
//   nothing above s) sets hi = s and the rest is goal runs at the middle of
//   (lo, hi].  s only grows and stays below hi, and goal runs never use the
//   forecast, so every pair settles.
// Every launch gets the full opts time limit; the node limit applies to the
// first run of strategy 1 only.
mcs_status mcs_solve_goals(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, int32_t strategy, void *workspace,
                           size_t bytes, void *stream, mcs_result *results,
                           int32_t *launches) {
    if (!results)
        return fail(MCS_E_INVALID, "results is NULL");
    for (int i = 0; i < count; i++)
        results[i].size = -1;
    if (strategy < 0 || strategy > 3)
        return fail(MCS_E_INVALID, "strategy must be 0 (top-down), 1 (bisection), 2 (dead-end, "
                                   "+1) or 3 (dead-end, doubling step)");
    const bool dead_strat = strategy >= 2;
    mcs_opts o1 = opts ? *opts : mcs_opts{};
    if (dead_strat && o1.deadend_nodes <= 0)
        return fail(MCS_E_INVALID, "strategies 2 and 3 need opts->deadend_nodes > 0");
    mcs_opts og = o1;
    if (strategy != 1)
        og.node_limit = 0;
    if (!dead_strat)
        og.deadend_nodes = 0, og.deadend_ratio = 0;
    mcs_plan *p = nullptr;
    mcs_status st = mcs_plan_create(count, G, H, &og, &p);
    if (st != MCS_OK)
        return st;
    struct PlanGuard {
        mcs_plan *p;
        ~PlanGuard() { mcs_plan_destroy(p); }
    } guard{p};
    st = mcs_plan_upload(p, workspace, bytes, stream);
    if (st != MCS_OK)
        return st;
    const int n = count;
    // kind: 0 settled, 1 plain run from start[i], 2 goal run at goal[i]
    std::vector<int> lo(n, 0), hi(n, 0), kind(n, 1), start(n, 0), goal(n, 0), step(n, 1);
    (void)mcs_plan_root_bounds(p, hi.data());
    std::vector<std::vector<int32_t>> mg(n), mh(n);
    std::vector<int64_t> nodes(n, 0);
    std::vector<double> tbest(n, 0.0), tproof(n, 0.0);
    std::vector<mcs_result> r(n);
    std::vector<std::vector<int32_t>> bg(n), bh(n);
    for (int i = 0; i < n; i++) {
        bg[i].assign(std::max(1, p->m[p->dev(i)]), 0);
        bh[i].assign(std::max(1, p->m[p->dev(i)]), 0);
        r[i] = mcs_result{};
        r[i].map_g = bg[i].data();
        r[i].map_h = bh[i].data();
        if (strategy == 0)
            kind[i] = 2;
    }
    double elapsed = 0.0;
    int runs = 0;
    bool limited = false;
    auto keep_map = [&](int i) {
        mg[i].assign(bg[i].begin(), bg[i].begin() + r[i].size);
        mh[i].assign(bh[i].begin(), bh[i].begin() + r[i].size);
    };
    auto settle = [&](int i) {
        kind[i] = 0;
        tproof[i] = elapsed;
    };
    auto bisect_next = [&](int i) {
        if (lo[i] >= hi[i]) {
            settle(i);
            return;
        }
        kind[i] = 2;
        goal[i] = strategy == 0 ? hi[i] : (lo[i] + 1 + hi[i] + 1) / 2;
        if (goal[i] <= lo[i])
            goal[i] = lo[i] + 1;
    };
    for (int i = 0; i < n; i++)
        if (lo[i] >= hi[i])
            settle(i);  // e.g. an empty graph: root bound 0
        else if (kind[i] == 2)
            bisect_next(i);
    std::vector<int32_t> lb(n), target(n), don(n), skip(n);
    for (;;) {
        bool any = false;
        for (int i = 0; i < n; i++) {
            skip[i] = kind[i] == 0;
            lb[i] = kind[i] == 1 ? start[i] : kind[i] == 2 ? goal[i] - 1 : 0;
            target[i] = kind[i] == 2 ? goal[i] : 0;
            don[i] = kind[i] == 1 && dead_strat ? 1 : 0;
            any = any || kind[i] != 0;
        }
        if (!any)
            break;
        if (elapsed >= o1.time_limit_s && o1.time_limit_s > 0) {
            limited = true;
            break;
        }
        st = apply_bounds(p, lb.data(), target.data(), don.data(), skip.data(), stream);
        if (st == MCS_OK)
            st = mcs_plan_run(p, stream);
        if (st == MCS_OK)
            st = mcs_plan_results(p, r.data(), stream);
        if (st < 0)
            return st;
        runs++;
        elapsed += p->last_ms / 1000.0;
        const bool stopped = p->h_glob.stop != 0;  // a time or node limit hit
        for (int i = 0; i < n; i++) {
            if (kind[i] == 0)
                continue;
            nodes[i] += r[i].nodes;
            const bool found = r[i].size > lb[i];
            if (found) {
                tbest[i] = elapsed - p->last_ms / 1000.0 + r[i].t_best_s;
                if (r[i].size > lo[i]) {
                    lo[i] = r[i].size;
                    keep_map(i);
                }
            }
            if (kind[i] == 2) {
                if (found) {
                    // reached: a mapping of at least the goal
                    if (strategy == 0)
                        hi[i] = lo[i];
                } else if (r[i].optimal) {
                    hi[i] = goal[i] - 1;  // refuted: nothing of size >= goal
                } else {
                    limited = true;  // this launch hit the time limit
                    kind[i] = 0;
                    continue;
                }
                bisect_next(i);
            } else if (r[i].optimal) {
                // a plain run finished: its best above start is the optimum,
                // and nothing above start means the raised bound is unreachable
                if (found)
                    hi[i] = lo[i];
                else
                    hi[i] = std::min(hi[i], start[i]);
                bisect_next(i);
            } else if (dead_strat && !stopped) {
                // forecast as a dead end: raise the bound (the best size so
                // far, or the bound this run already started from) by the step
                const int cur = std::max(lo[i], start[i]);
                const int s = std::min(cur + step[i], hi[i] - 1);
                if (strategy == 3)
                    step[i] *= 2;
                if (s <= cur)
                    bisect_next(i);  // no room left to raise it: settle by goals
                else
                    start[i] = s;
            } else if (strategy == 1 && runs == 1 && stopped) {
                // the node-limited first run of strategy 1: bisect from lo
                bisect_next(i);
            } else {
                limited = true;
                kind[i] = 0;
            }
        }
        if (strategy == 1 && runs == 1)
            p->sp.node_limit = 0;
    }
    for (int i = 0; i < n; i++) {
        mcs_result &o = results[i];
        o.size = lo[i];
        o.optimal = (lo[i] >= hi[i]) ? 1 : 0;
        o.nodes = nodes[i];
        o.t_best_s = tbest[i];
        o.t_proof_s = o.optimal ? tproof[i] : 0.0;
        for (int j = 0; j < lo[i]; j++) {
            if (o.map_g)
                o.map_g[j] = mg[i][j];
            if (o.map_h)
                o.map_h[j] = mh[i][j];
        }
    }
    if (launches)
        *launches = runs;
    bool all = true;
    for (int i = 0; i < n; i++)
        all = all && results[i].optimal;
    return (all && !limited) ? MCS_OK : MCS_LIMIT;
}

size_t mcs_workspace_size(int32_t count, const mcs_graph *G, const mcs_graph *H,
                          const mcs_opts *opts) {
    mcs_plan *p = nullptr;
    if (mcs_plan_create(count, G, H, opts, &p) != MCS_OK)
        return 0;
    size_t b = p->ws_bytes;
    mcs_plan_destroy(p);
    return b;
}

mcs_status mcs_solve_batch(int32_t count, const mcs_graph *G, const mcs_graph *H,
                           const mcs_opts *opts, void *workspace, size_t bytes, void *stream,
                           mcs_result *results) {
    if (results && count > 0)
        for (int i = 0; i < count; i++)
            results[i].size = -1;
    if (!results)
        return fail(MCS_E_INVALID, "results is NULL");
    mcs_plan *p = nullptr;
    mcs_status s = mcs_plan_create(count, G, H, opts, &p);
    if (s != MCS_OK)
        return s;
    s = mcs_plan_upload(p, workspace, bytes, stream);
    if (s == MCS_OK)
        s = mcs_plan_run(p, stream);
    if (s == MCS_OK)
        s = mcs_plan_results(p, results, stream);
    if (s < 0)
        for (int i = 0; i < count; i++)
            results[i].size = -1;
    mcs_plan_destroy(p);
    return s;
}

mcs_status mcs_solve_batch_static(int32_t count, const mcs_graph *G, const mcs_graph *H,
                                  const mcs_opts *opts, void *stream, mcs_result *results) {
    if (!results)
        return fail(MCS_E_INVALID, "results is NULL");
    for (int i = 0; i < count; i++)
        results[i].size = -1;
    if (opts && opts->tuning && opts->tuning->use_graph)
        return fail(MCS_E_INVALID, "the static-scratch entry does not run the HIP graph mode "
                                   "(it stages through pinned host memory)");
    size_t cap = 0;
    int herr = 0;
    uint8_t *scratch = (uint8_t *)mcs_internal_static_scratch(&cap, &herr);
    if (!scratch)
        return fail(MCS_E_DEVICE, "cannot look up the static scratch's device address (HIP "
                                  "error " + std::to_string(herr) + ")");
    mcs_plan *p = nullptr;
    mcs_status s = mcs_plan_create(count, G, H, opts, &p);
    if (s != MCS_OK)
        return s;
    struct PlanGuard {
        mcs_plan *p;
        ~PlanGuard() { mcs_plan_destroy(p); }
    } guard{p};
    if (p->ws_bytes > cap)
        return fail(MCS_E_WORKSPACE, "the batch needs " + std::to_string(p->ws_bytes) +
                                         " bytes of workspace, more than the " +
                                         std::to_string(cap) +
                                         "-byte static scratch: use mcs_solve_batch, or "
                                         "fewer wavefronts per CU");
    p->no_events = true;
    s = mcs_plan_upload(p, scratch, cap, stream);
    if (s == MCS_OK)
        s = mcs_plan_run(p, stream);
    if (s == MCS_OK)
        s = mcs_plan_results(p, results, stream);
    if (s < 0)
        for (int i = 0; i < count; i++)
            results[i].size = -1;
    return s;
}

mcs_status mcs_solve(const mcs_graph *G, const mcs_graph *H, const mcs_opts *opts, void *workspace,
                     size_t bytes, void *stream, mcs_result *result) {
    return mcs_solve_batch(1, G, H, opts, workspace, bytes, stream, result);
}

}  // extern "C"
