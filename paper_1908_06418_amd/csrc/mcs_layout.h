// Device-side data layout shared by the host driver (mcs_host.cpp) and the
// search kernels (mcs_search.hip).
#pragma once
#include <stdint.h>

namespace mcs {

// One instance, as the kernels see it.  Vertices are already in descending
// degree order; adjacency rows and root classes live in separate arrays.
struct DevInst {
    uint8_t nG, nH, K0, pad;
    uint32_t cls_off;  // first root class in the root-class array
    uint32_t map_off;  // first mapping pair of this instance's per-size slots
    int32_t lb;        // initial incumbent size (0: none)
    int32_t target;    // > 0: stop this instance once a mapping of this size is found
    int32_t inc_slot;  // incumbent word this instance reads and raises (its own
                       // index, or its portfolio twin's: twins share one)
    int32_t twin;      // the same pair entered under another vertex order, or -1;
                       // once either twin's search is finished the other stops
    int32_t dead_on;   // 1: this run may give the instance up as a dead end
};

// The node queue is sharded into one ring per XCD (workgroup i runs on XCD
// i mod 8): a wavefront donates into its own XCD's ring and takes from it
// first, stealing from the other rings only when its own is empty.
constexpr int kRings = 8;

struct RingCtl {
    unsigned long long head;  // next ticket to take
    uint8_t pad_head[120];
    unsigned long long tail;  // next ticket to fill
    uint8_t pad_tail[120];
};

// Flags a wavefront polls, one copy per XCD on a line of its own: they are
// written once per launch (by the wavefront that stops or ends the search,
// into every copy), so polling them never contends with counter updates.
constexpr unsigned kFlagStop = 1;  // a limit was hit or a capacity check fired
constexpr unsigned kFlagDone = 2;  // no work unit is left

struct XcdCtl {
    unsigned flag;
    uint8_t pad[124];
};

// Counters shared by every wavefront of a launch.  The ones wavefronts
// update each sit on a cache line of their own.
struct DevGlobals {
    RingCtl ring[kRings];
    XcdCtl xcd[kRings];
    int open_total;                 // work units alive: instances not yet claimed,
                                    // queued nodes and busy wavefronts
    unsigned stop;                  // 1: a limit was hit (reported to the host)
    uint8_t pad_state[120];
    unsigned next_inst;             // next instance whose root is not yet taken
    uint8_t pad_next[124];
    unsigned long long t0;          // earliest wavefront start (realtime ticks)
    unsigned long long node_total;  // nodes flushed so far (for the node limit)
    unsigned error;                 // nonzero: a capacity check fired
    int pad0;
    unsigned long long batches;     // statistics
    unsigned long long children;
    unsigned long long lane_slots;
    unsigned long long donations;
    unsigned long long pops;
    unsigned long long busy_ticks;  // realtime ticks wavefronts spent searching
    unsigned long long hbm_frames;  // frames placed in the HBM part of a class stack
    unsigned long long sleep_ticks; // realtime ticks idle wavefronts spent sleeping
    unsigned long long pushed_classes;  // classes in the frames pushed onto LDS stacks
    unsigned long long node_classes;    // classes split, summed over the matched
                                        // children counted as nodes (first
                                        // evaluations only)
    int max_stack;                  // most classes any wavefront's stack held
    int pad1;
};

struct SearchParams {
    const DevInst *inst;
    const void *adj;      // [count][R][NB] words, R = 2 (G, H) or 4 (G out, H out, G in, H in)
    const void *rootcls;  // [sum K0] (L, R) word pairs
    int *inc;             // [count] incumbent size
    int *open;            // [count] live work units of the instance (1 while unclaimed)
    unsigned long long *nodes;    // [count]
    unsigned long long *t_best;   // [count] (size << 48) | (realtime & 2^48-1)
    unsigned long long *t_proof;  // [count] realtime ticks when open reached 0
    unsigned long long *best_nodes;  // [count] the instance's node count when its
                                     // incumbent was last raised
    int *dead;                    // [count] 1: given up as a dead end
    uint16_t *maps;               // per instance, per size s: s pairs (g | h << 8)
    DevGlobals *g;
    unsigned long long *seq;      // [kRings][ring_slots] queue slot sequence numbers
    uint8_t *slots;               // [kRings][ring_slots][slot_bytes]
    int count;
    int ring_slots;               // slots per ring (a power of two)
    int slot_bytes;
    int cap_classes;      // LDS class capacity of one wavefront's stack
    int frames;           // frame headers per wavefront (largest min(nG, nH) + 1)
    int lds_per_wave;     // bytes
    int cmax;             // children per batch (1, 2, 4, 8)
    int donate_low;       // records a busy wavefront keeps queued in its XCD's ring (< 0: never donate)
    int donate_depth;     // only frames with |M| <= this are donated
    int check_interval;
    int backoff_max;      // most sleeps (of about 3.4 us) between an idle wavefront's polls
    int reprune;
    int single_wave;
    const uint16_t *policy;  // half-precision policy parameters, or null
    int policy_depth;        // policy orders frames with |M| <= this
    int policy_mode;         // bit 0: policy picks v; bit 1: policy orders partners
    int policy_levels;       // LDS partner-order lists per wavefront (0 without policy)
    unsigned long long limit_ticks;  // time limit in realtime ticks
    long long node_limit;            // 0: none
    long long dead_abs;              // dead-end forecast (instances with dead_on): more
                                     // than this many nodes since the last improvement
                                     // (0: never)
    long long dead_rel;              // ... and more than this many times the nodes that
                                     // led to the last improvement (0: absolute only)
    uint8_t *hstack;                 // HBM class stacks, or null: [waves][hstack_stride]
                                     // (128-bit rows), [waves][searches][hstack_stride]
                                     // (segments: the part above the LDS part)
    long long hstack_stride;         // bytes per stack (0: no HBM part)
    int seg_log;                     // segmented kernel: 2^seg_log lanes per search (0: one
                                     // search per wavefront)
    int seg_bytes;                   // segmented kernel: LDS bytes per search (seg_layout)
    int arows;                       // segmented kernel: adjacency rows kept per graph in LDS
    int pad_seg;
};

struct ResetParams {
    const DevInst *inst;
    int *inc;
    int *open;
    unsigned long long *nodes;
    unsigned long long *t_best;
    unsigned long long *t_proof;
    unsigned long long *best_nodes;
    int *dead;
    DevGlobals *g;
    unsigned long long *seq;
    int count;
    int ring_slots;
};

// Words of one frame header in LDS (one 32-bit word per field, padded).
// Rows of 128 bits need two more words for the remaining-partner mask, rows
// of 256 bits six.
constexpr int kHdrWords = 12;
constexpr int kHdrWordsWide = 14;
constexpr int kHdrWords256 = 18;
inline constexpr int hdr_words(int word_bytes) {
    return word_bytes > 16 ? kHdrWords256 : word_bytes > 8 ? kHdrWordsWide : kHdrWords;
}

// Record of a donated node in the queue: a header (32 bytes, 48 with
// 256-bit rows), the mapping (NB pairs of bytes) and the classes.
constexpr int kRecHeader = 32;
inline constexpr int rec_header(int word_bytes) { return word_bytes > 16 ? 48 : kRecHeader; }

template <typename W>
constexpr int bits_of() { return 8 * (int)sizeof(W); }

template <typename W>
constexpr int rec_map_off() { return rec_header((int)sizeof(W)); }

template <typename W>
constexpr int rec_cls_off() { return rec_header((int)sizeof(W)) + 2 * bits_of<W>(); }

// LDS of one wavefront, in this order, each part 16-byte aligned:
//   classes   [cap_classes + 1] (L, R) word pairs; the last is a trash slot
//             that lanes with nothing to store write to, so the stores need
//             no exec-mask branches (cap_classes = -1: the classes live
//             elsewhere, as they do in HBM for 128-bit rows)
//   adjacency [R][NB] words (R = 4 directed, 2 undirected; with rows wider
//             than 64 bits only H's rows, R = 2 or 1)
//   mapping   [NB] byte pairs
//   headers   [frames][hdr_words] frame headers, one 32-bit word per field
//   orders    [policy levels][64] partner order of policy-ordered frames
struct LdsLayout {
    int cls, adj, map, hdr, ord, total;
};

inline constexpr int align16(int x) { return (x + 15) & ~15; }

inline constexpr LdsLayout lds_layout(int word_bytes, int directed, int cap_classes,
                                      int frames, int policy_levels = 0) {
    int nb = 8 * word_bytes;
    int rows = (directed ? 4 : 2) / (word_bytes > 8 ? 2 : 1);
    int hdr_bytes = 4 * hdr_words(word_bytes);
    LdsLayout L{0, 0, 0, 0, 0, 0};
    L.cls = 0;
    L.adj = align16((cap_classes + 1) * 2 * word_bytes);
    L.map = align16(L.adj + rows * nb * word_bytes);
    L.hdr = align16(L.map + 2 * nb);
    L.ord = align16(L.hdr + frames * hdr_bytes);
    L.total = align16(L.ord + policy_levels * 64);
    return L;
}

// LDS of one search of the segmented kernel (one per lane segment), each
// part 16-byte aligned:
//   classes   [cap_classes] (L, R) word pairs
//   adjacency [R][arows] words of H: out-rows (and in-rows if directed);
//             rows past arows are never read: arows is at least the
//             largest vertex count of the batch.  (The search keeps the
//             G rows of v in registers, loaded from HBM once per frame.)
//   mapping   [frames] byte pairs, one per depth
//   headers   [frames] frame headers of two 32-bit words
struct SegLayout {
    int cls, adj, map, hdr, total;
};

inline constexpr SegLayout seg_layout(int word_bytes, int directed, int cap_classes, int arows,
                                      int frames) {
    int rows = directed ? 2 : 1;
    SegLayout L{0, 0, 0, 0, 0};
    L.cls = 0;
    L.adj = align16(cap_classes * 2 * word_bytes);
    L.map = align16(L.adj + rows * arows * word_bytes);
    L.hdr = align16(L.map + 2 * frames);
    L.total = align16(L.hdr + frames * 8);
    return L;
}

inline int slot_bytes_for(int word_bytes, int mmax) {
    int b = rec_header(word_bytes) + 2 * 8 * word_bytes + mmax * 2 * word_bytes;
    return (b + 63) & ~63;
}

}  // namespace mcs
