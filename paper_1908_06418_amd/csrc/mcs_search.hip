// McSplit search kernels for gfx950 (CDNA4, wave64).
//
// The work of one search node is the paper's Solve body (Sec. II.B,
// Algorithm 1): split every label class by adjacency to v (G side) and to w
// (H side) -- filterDomain -- and bound the child with Eq. 1,
//     bound = |M| + sum over classes of min(|L|, |R|),
// pruning it when the bound cannot beat the incumbent.
//
// GPU mapping (ours, not the paper's CUDA design):
//   * One wavefront runs one depth-first search at a time.  Classes are
//     bitsets (L, R) of one word each (32-bit rows for graphs of at most 32
//     vertices, 64-bit up to 64, 128-bit up to 128, 256-bit up to 254);
//     lane k holds class k.  A node has at most min(|V_G|, |V_H|) classes,
//     so one wave64 holds all of them up to 64 vertices; with wider rows a
//     frame of more than 64 classes puts class 64q + k in slot q of lane k.
//   * A batch evaluates up to 8 sibling children at once: lanes are split in
//     segments of S = 8/16/32/64 lanes, each segment a copy of the classes and
//     its own w.  Split, popcounts and the min() of Eq. 1 are per lane; the
//     per-segment sum is a DPP reduction.  Prune decisions are wave-uniform,
//     so the bound test never diverges.
//   * A surviving child's classes are compacted (ballot + mbcnt) into the
//     wave's LDS stack.  Stack frames hold the classes of each open node on
//     the current path; the "v unmatched" child rewrites its parent frame in
//     place, so m(m+1)/2 classes (m = min(|V_G|, |V_H|)) is the worst case.
//     The host may size the stack below that to fit more wavefronts per CU;
//     a child that does not fit goes to the node queue as a fresh record.
//   * Frame headers are one 32-bit word per field, written from the lanes of
//     one register (v_writelane) and read back by readlane; stores that only
//     some lanes have data for send the others to a trash slot instead of
//     branching on the exec mask (the scalar unit is the busiest one).
//   * Work sharing: bounded lock-free rings of node records in HBM (Vyukov
//     sequence numbers), one per XCD.  A busy wave keeps its XCD's ring
//     stocked: when its periodic check finds fewer than a few records
//     waiting, it donates the shallowest frame that still has unexplored
//     children (as the paper's thread pool hands out shallow tasks first).
//     Idle waves take records (their own ring first, then steal) or new
//     instance roots.  The paper's shared loop index becomes the donated
//     frame's remaining-children mask.
//   * Incumbents: one int per instance, atomicMax at agent scope; the mapping
//     of size s is written to a per-size slot by the unique wave that raised
//     the incumbent to s.
//   * Termination: a count of live work units (queued records plus busy
//     waves), per instance and in total; the wave that ends the last unit
//     raises a done flag (one copy per XCD, so polling it is cheap); every
//     wave also leaves at the time limit, so the grid always drains.
#include "mcs_device.h"
#include "mcs_policy.h"

namespace mcs {

// ---- one wavefront's search ------------------------------------------------

template <typename W, bool DIR, bool POL>
struct Searcher {
    static constexpr int NB = bits_of<W>();  // vertices per row word
    static constexpr int NR = DIR ? 4 : 2;   // adjacency row sets per instance
    static constexpr int Q = NB > 64 ? NB / 64 : 1;  // class slots per lane
    static constexpr int HW = hdr_words((int)sizeof(W));  // header words per frame
    static_assert(!(POL && Q > 1), "the policy scorer takes one vertex per lane");

    const SearchParams &P;  // a copy in LDS: cold fields are read when needed
    int cmax, cap_classes, check_interval, reprune;  // hot knobs, kept in registers
    int lane;
    W *sadj;        // [NR][NB]: G rows, H rows (out), then G, H in-rows; with
                    // rows wider than 64 bits only H's: [NR / 2][NB] (out, in)
    const W *gadj;  // (rows wider than 64 bits) the instance's rows in HBM, for v's G rows
    uint16_t *smap; // [NB] current path: g | h << 8
    int *shdr;      // [NB + 1][HW]
    Cls<W> *scls;   // [cap_classes + 1] (LDS; HBM with 128-bit rows)

    uint8_t *sord;  // [policy levels][64]: partner order of policy-ordered frames
    int inst, map_off, nG, nH, target;
    int inc_slot, twin;  // shared incumbent word; portfolio twin (or -1)
    int dead_on;         // the instance may be given up as a dead end
    // top frame, wave-uniform
    int t, base, K, d, v, sel, bound, flags, lsel, rsel;
    W rrem;
    int logS;
    // this lane's copy of class (lane mod S) of the top frame, and in a
    // frame of more than 64 classes (S = 64), of class lane + 64q in slot q
    // (cLh[q - 1], cRh[q - 1])
    W cL, cR;
    W cLh[Q > 1 ? Q - 1 : 1], cRh[Q > 1 ? Q - 1 : 1];
    int inc;
    bool stop;
    bool roots_left;  // false once every instance root has been claimed
    int my_ring;      // this workgroup's XCD ring
    int steal_from;   // the other ring tried next when idle
    int d0;           // depth of the unit's first frame (the shallowest)
    int since_check;
    unsigned long long t_start, pend_nodes, n_batches, n_children, n_lanes, n_don, n_pops, n_busy;
    unsigned long long n_sleep;
    int max_used;  // most classes this wavefront's stack has held
    // per-step counts since the last fold into the 64-bit totals (at most
    // check_interval steps, so 32 bits cannot overflow)
    uint32_t c_nodes, c_batches, c_children, c_lanes, c_ncls;
    // classes in frames pushed since the last fold (the host turns this and
    // the batch counts into the bytes the search moves through LDS)
    uint32_t c_pushed;
    unsigned long long n_pushed, n_ncls;

    __device__ Searcher(const SearchParams &p, uint8_t *lds, int wave) : P(p) {
        lane = lane_id();
        cmax = sc(p.cmax);
        cap_classes = sc(p.cap_classes);
        check_interval = sc(p.check_interval);
        reprune = sc(p.reprune);
        // with 128-bit rows the class stack is this wavefront's slice of HBM
        // (the worst case, up to 264 KB, does not fit in LDS)
        const LdsLayout L = lds_layout((int)sizeof(W), DIR ? 1 : 0, Q == 1 ? p.cap_classes : -1,
                                       p.frames, p.policy_levels);
        if constexpr (Q == 1)
            scls = (Cls<W> *)(lds + L.cls);
        else
            scls = (Cls<W> *)(p.hstack + (size_t)wave * (size_t)p.hstack_stride);
        sadj = (W *)(lds + L.adj);
        gadj = (const W *)p.adj;
        smap = (uint16_t *)(lds + L.map);
        shdr = (int *)(lds + L.hdr);
        sord = lds + L.ord;
        inst = -1;
        map_off = 0;
        nG = nH = 1;
        target = 0;
        inc_slot = 0;
        twin = -1;
        dead_on = 0;
        stop = false;
        roots_left = true;
        my_ring = (int)(blockIdx.x & (kRings - 1));
        steal_from = my_ring;
        d0 = 0;
        since_check = 0;
        pend_nodes = n_batches = n_children = n_lanes = n_don = n_pops = n_busy = 0;
        c_nodes = c_batches = c_children = c_lanes = c_pushed = c_ncls = 0;
        n_pushed = n_ncls = 0;
        n_sleep = 0;
        max_used = 0;
        inc = 0;
        t = -1;
    }

    // Sets flag bits in every XCD's copy; a stop is also recorded in the
    // word the host reads back.  Safe to call from lane 0 alone.
    __device__ void raise_flag(unsigned bits) {
        if (lane == 0) {
            if (bits & kFlagStop)
                __hip_atomic_store(&P.g->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 0; k < kRings; ++k)
                __hip_atomic_fetch_or(&P.g->xcd[k].flag, bits, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // code 1: a capacity check that cannot fire unless there is a bug;
    // code 2: the node queue was full when a child had to be queued.
    __device__ void fail(unsigned code) {
        if (lane == 0)
            __hip_atomic_store(&P.g->error, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        raise_flag(kFlagStop);
        stop = true;
    }

    // Orders a wavefront's own stack traffic between its lanes.
    __device__ void sync() {
        if constexpr (Q == 1)
            wave_sync();
        else
            wave_sync_global();
    }

    // Slot q of this lane's classes.  A constant q names a register; a
    // wave-uniform q selects (register arrays are never indexed at run time).
    __device__ W slotL(int q) const {
        W x = cL;
#pragma unroll
        for (int j = 1; j < Q; ++j)
            x = pick(q == j, cLh[j - 1], x);
        return x;
    }
    __device__ W slotR(int q) const {
        W x = cR;
#pragma unroll
        for (int j = 1; j < Q; ++j)
            x = pick(q == j, cRh[j - 1], x);
        return x;
    }

    // -- frame registers -----------------------------------------------------

    __device__ void load_regs() {
        if constexpr (Q == 1) {
            logS = K <= 8 ? 3 : K <= 16 ? 4 : K <= 32 ? 5 : 6;
            const int k = lane & ((1 << logS) - 1);
            const bool in = k < K;
            const Cls<W> c = scls[base + (in ? k : 0)];  // (no exec-mask branch)
            cL = in ? c.L : (W)0;
            cR = in ? c.R : (W)0;
        } else {
            // segments as with one class per lane; only a frame of more
            // than 64 classes (S = 64) puts classes 64q.. in slot q
            logS = K <= 8 ? 3 : K <= 16 ? 4 : K <= 32 ? 5 : 6;
            const int S = 1 << logS;
            const int k = lane & (S - 1);
            const bool in0 = k < K;
            const Cls<W> c0 = ld_cls(scls + base + (in0 ? k : 0));
            cL = pick(in0, c0.L, (W)0);
            cR = pick(in0, c0.R, (W)0);
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                cLh[q - 1] = (W)0;
                cRh[q - 1] = (W)0;
                if (K > 64 * q) {
                    const bool in = k + 64 * q < K;
                    const Cls<W> c = ld_cls(scls + base + (in ? k + 64 * q : 0));
                    cLh[q - 1] = pick(in, c.L, (W)0);
                    cRh[q - 1] = pick(in, c.R, (W)0);
                }
            }
        }
    }

    // selectLabelClass + selectVertex: the class with the smallest
    // max(|L|, |R|), ties to the smallest vertex of L; v = that vertex.
    __device__ void select() {
        if constexpr (Q > 1) {
            select_wide();
            return;
        }
        uint32_t key = 0xFFFFFFFFu;
        if (lane < K) {
            int nl = popc(cL), nr = popc(cR);
            key = ((uint32_t)(nl > nr ? nl : nr) << 8) | (uint32_t)ctz(cL);
        }
        uint32_t mk = seg0_min(key, logS);
        int who = ctz((uint64_t)ballot(key == mk));
        sel = who;
        v = (int)(mk & 0xFF);
        rrem = rl(cR, who);
        lsel = popc(rl(cL, who));
        rsel = popc(rrem);
        flags &= ~kFlagOrdered;
        if constexpr (POL) {
            if (d <= P.policy_depth && t < P.policy_levels) {
                // learned choice of v within the class, and of the partners' order
                const int mode = P.policy_mode;
                if (mode & 1) {
                    float sg = policy_score(0, rl(cL, who));
                    v = argmax_lane(sg, rl(cL, who));
                }
                if (mode & 2)
                    order_partners(rrem);
            }
        }
    }

    // select() with Q class slots per lane (class lane + qS in slot q; slots
    // past the first are used only when S = 64).  L sets are disjoint, so
    // keys are distinct.
    __device__ void select_wide() {
        const int S = 1 << logS;
        uint32_t key[Q];
        uint32_t kmin = 0xFFFFFFFFu;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            key[q] = 0xFFFFFFFFu;
            if (lane < S && lane + q * S < K) {
                const W l = slotL(q), r = slotR(q);
                int nl = popc(l), nr = popc(r);
                key[q] = ((uint32_t)(nl > nr ? nl : nr) << 8) | (uint32_t)ctz(l);
            }
            kmin = umin(kmin, key[q]);
        }
        const uint32_t mk = seg0_min(kmin, logS);
        int hq = 0;
#pragma unroll
        for (int q = 1; q < Q; ++q)
            hq = key[q] == mk ? q : hq;
        const int who = ctz((uint64_t)ballot(kmin == mk));
        hq = rl(hq, who);
        sel = who + hq * S;
        v = (int)(mk & 0xFF);
        rrem = rl(slotR(hq), who);
        lsel = popc(rl(slotL(hq), who));
        rsel = popc(rrem);
        flags &= ~kFlagOrdered;
    }

    // -- learned branching policy ----------------------------------------------
    // Scores of the candidate vertices `cand` of one side, from the 16
    // features the policy reference defines and the half-precision network:
    // lane u returns the score of vertex u.  One lane per hidden unit (both
    // hidden layers are 64 wide) and one candidate at a time: the features
    // are wave-uniform, layer 1 is 16 multiply-adds per lane, layer 2 takes
    // every lane's layer-1 output by readlane, and the output is a wave sum.
    // This keeps the scorer's registers few, so a policy kernel runs as many
    // wavefronts per CU as a plain one; the scorer itself runs only at
    // shallow frames.
    __device__ float policy_score(int side, W cand) {
        const int off = side ? NB : 0;
        const int n = side ? nH : nG;
        const float inv = 1.f / (float)(n > 0 ? n : 1);
        // class lanes: this side's set and the class-size bucket (8-bit field)
        W mine = 0;
        int bsh = 0;
        if (lane < K) {
            Cls<W> c = scls[base + lane];
            const int nl = popc(c.L), nr = popc(c.R);
            const int m = nl < nr ? nl : nr;
            const int bq = m <= 1 ? 0 : m == 2 ? 1 : m <= 4 ? 2 : m <= 8 ? 3 : m <= 16 ? 4 : 5;
            mine = side ? c.R : c.L;
            bsh = 8 * bq;
        }
        // largest degree among the candidates
        const int ul = lane & (NB - 1);
        W rowl = sadj[off + ul];
        if (DIR)
            rowl |= sadj[2 * NB + off + ul];
        const bool is_cand = lane < NB && ((cand >> ul) & 1);
        const int dmax = (int)~wave_min(~(uint32_t)(is_cand ? popc(rowl) : 0));
        // this lane's hidden unit
        const uint16_t *w = P.policy;
        float w1[kPolicyF];
#pragma unroll
        for (int f = 0; f < kPolicyF; ++f)
            w1[f] = hf(w[kOffW1 + lane * kPolicyF + f]);
        const float b1 = hf(w[kOffB1 + lane]), b2 = hf(w[kOffB2 + lane]);
        const float w3 = hf(w[kOffW3 + lane]), b3 = hf(w[kOffB3]);
        const uint4 *w2 = (const uint4 *)(w + kOffW2 + lane * kPolicyH);  // 16-byte aligned
        float out = 0.f;
        for (W rest = cand; rest; rest &= rest - 1) {
            const int u = sc((int)ctz(rest));
            W row = sadj[off + u];
            if (DIR)
                row |= sadj[2 * NB + off + u];
            row = sc(row);
            const int deg = popc(row);
            // neighbours of u per class, summed per size bucket (each sum is
            // at most deg < 64, so 8-bit fields cannot carry)
            const unsigned long long packed = (unsigned long long)popc(row & mine) << bsh;
            const int lo = wave_sum((int)(uint32_t)packed);
            const int hi = wave_sum((int)(uint32_t)(packed >> 32));
            float x[kPolicyF];
            x[0] = deg * inv;
            x[1] = lsel * inv;
            x[2] = rsel * inv;
            x[3] = d * inv;
            x[4] = K * inv;
            int tot = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int cq = q < 4 ? (lo >> (8 * q)) & 0xFF : (hi >> (8 * (q - 4))) & 0xFF;
                x[6 + q] = cq * inv;
                tot += cq;
            }
            x[5] = tot * inv;
            x[12] = (float)side;
            x[13] = deg == dmax ? 1.f : 0.f;
            x[14] = 0.f;
            x[15] = 1.f;
            float h1 = b1;
#pragma unroll
            for (int f = 0; f < kPolicyF; ++f)
                h1 += w1[f] * x[f];
            h1 = h1 > 0.f ? h1 : 0.f;
            float a2 = b2;
#pragma unroll 1
            for (int c = 0; c < kPolicyH / 8; ++c) {
                const uint4 q = w2[c];
                const uint32_t pk[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    a2 += hf((uint16_t)(pk[e] & 0xFFFFu)) * rlf(h1, 8 * c + 2 * e);
                    a2 += hf((uint16_t)(pk[e] >> 16)) * rlf(h1, 8 * c + 2 * e + 1);
                }
            }
            const float z = b3 + fwave_sum(w3 * (a2 > 0.f ? a2 : 0.f));
            out = lane == u ? z : out;
        }
        return out;
    }

    // Highest-scoring candidate lane (lowest index among equal scores).
    __device__ int argmax_lane(float score, W cand) {
        const bool is_cand = lane < NB && ((cand >> (lane & (NB - 1))) & 1);
        // order-preserving map of floats to unsigned ints
        uint32_t b = __float_as_uint(score);
        uint32_t key = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
        key = is_cand ? key : 0u;
        uint32_t best = ~wave_min(~key);
        return ctz((uint64_t)ballot(is_cand && key == best));
    }

    // sord[t][r] = the r-th best partner among cand (ties by index).
    __device__ void order_partners(W cand) {
        float s = policy_score(1, cand);
        const bool is_cand = lane < NB && ((cand >> (lane & (NB - 1))) & 1);
        uint32_t b = __float_as_uint(s);
        uint32_t key = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
        int rank = 0;
        W rest = cand;
        while (rest) {
            int c = ctz(rest);
            rest &= rest - 1;
            uint32_t kc = rl(key, c);
            rank += (kc > key || (kc == key && c < lane)) ? 1 : 0;
        }
        if (is_cand)
            sord[t * 64 + rank] = (uint8_t)lane;
        sync();
        flags |= kFlagOrdered;
    }

    __device__ void save_top() {
        // lane f of x takes field f (one asm block: no hazard padding
        // between the writes, which depend on nothing but their operands)
        int x = 0;
        const int lo = (int)(uint32_t)rrem;
        const int hi = sizeof(W) >= 8 ? (int)(uint32_t)((uint64_t)rrem >> 32) : 0;
        static_assert(kHRremLo == 0 && kHRremHi == 1 && kHBase == 2 && kHK == 3 && kHD == 4 &&
                          kHV == 5 && kHSel == 6 && kHBound == 7 && kHFlags == 8 &&
                          kHLsel == 9 && kHRsel == 10,
                      "header field order");
        asm volatile(
            "v_writelane_b32 %0, %1, 0\n\t"
            "v_writelane_b32 %0, %2, 1\n\t"
            "v_writelane_b32 %0, %3, 2\n\t"
            "v_writelane_b32 %0, %4, 3\n\t"
            "v_writelane_b32 %0, %5, 4\n\t"
            "v_writelane_b32 %0, %6, 5\n\t"
            "v_writelane_b32 %0, %7, 6\n\t"
            "v_writelane_b32 %0, %8, 7\n\t"
            "v_writelane_b32 %0, %9, 8\n\t"
            "v_writelane_b32 %0, %10, 9\n\t"
            "v_writelane_b32 %0, %11, 10"
            : "+v"(x)
            : "s"(lo), "s"(hi), "s"(base), "s"(K), "s"(d), "s"(v), "s"(sel), "s"(bound),
              "s"(flags), "s"(lsel), "s"(rsel));
        if constexpr (sizeof(W) == 16) {
            static_assert(kHRrem2 == 11 && kHRrem3 == 12, "header field order");
            const int w2 = (int)(uint32_t)((u128)rrem >> 64);
            const int w3 = (int)(uint32_t)((u128)rrem >> 96);
            asm volatile(
                "v_writelane_b32 %0, %1, 11\n\t"
                "v_writelane_b32 %0, %2, 12"
                : "+v"(x)
                : "s"(w2), "s"(w3));
        } else if constexpr (sizeof(W) == 32) {
            static_assert(kHRrem2 == 11 && kHRrem7 == 16, "header field order");
            const int w2 = (int)(uint32_t)rrem.w[1], w3 = (int)(uint32_t)(rrem.w[1] >> 32);
            const int w4 = (int)(uint32_t)rrem.w[2], w5 = (int)(uint32_t)(rrem.w[2] >> 32);
            const int w6 = (int)(uint32_t)rrem.w[3], w7 = (int)(uint32_t)(rrem.w[3] >> 32);
            asm volatile(
                "v_writelane_b32 %0, %1, 11\n\t"
                "v_writelane_b32 %0, %2, 12\n\t"
                "v_writelane_b32 %0, %3, 13\n\t"
                "v_writelane_b32 %0, %4, 14\n\t"
                "v_writelane_b32 %0, %5, 15\n\t"
                "v_writelane_b32 %0, %6, 16"
                : "+v"(x)
                : "s"(w2), "s"(w3), "s"(w4), "s"(w5), "s"(w6), "s"(w7));
        }
        // lanes past the last field all store into the header's padding word
        shdr[t * HW + (lane < HW ? lane : HW - 1)] = x;
    }

    // One field of frame i's header, as a scalar.
    __device__ int hdr(int i, int f) const { return sc(shdr[i * HW + f]); }
    __device__ W hdr_rrem(int i) const {
        if constexpr (sizeof(W) == 32) {
            uint64_t ws[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                ws[k] = (uint64_t)(uint32_t)hdr(i, rrem_field(2 * k)) |
                        ((uint64_t)(uint32_t)hdr(i, rrem_field(2 * k + 1)) << 32);
            return from_words<W>(ws);
        }
        W r = (W)(uint32_t)hdr(i, kHRremLo);
        if constexpr (sizeof(W) >= 8)
            r |= (W)(uint32_t)hdr(i, kHRremHi) << 32;
        if constexpr (sizeof(W) == 16) {
            r |= (W)(uint32_t)hdr(i, kHRrem2) << 64;
            r |= (W)(uint32_t)hdr(i, kHRrem3) << 96;
        }
        return r;
    }

    __device__ void read_hdr(int i) {
        const int x = shdr[i * HW + (lane < HW ? lane : 0)];
        W r = (W)(uint32_t)rl(x, kHRremLo);
        if constexpr (sizeof(W) == 32) {
            uint64_t ws[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                ws[k] = (uint64_t)(uint32_t)rl(x, rrem_field(2 * k)) |
                        ((uint64_t)(uint32_t)rl(x, rrem_field(2 * k + 1)) << 32);
            r = from_words<W>(ws);
        }
        if constexpr (sizeof(W) >= 8 && sizeof(W) <= 16)
            r |= (W)(uint32_t)rl(x, kHRremHi) << 32;
        if constexpr (sizeof(W) == 16) {
            r |= (W)(uint32_t)rl(x, kHRrem2) << 64;
            r |= (W)(uint32_t)rl(x, kHRrem3) << 96;
        }
        rrem = r;
        base = rl(x, kHBase);
        K = rl(x, kHK);
        d = rl(x, kHD);
        v = rl(x, kHV);
        sel = rl(x, kHSel);
        bound = rl(x, kHBound);
        flags = rl(x, kHFlags);
        lsel = rl(x, kHLsel);
        rsel = rl(x, kHRsel);
    }

    // -- instances -------------------------------------------------------------

    __device__ void set_instance(int i) {
        if (i != inst) {
            const W *src = (const W *)P.adj + (size_t)i * NR * NB;
            if constexpr (Q == 1) {
                for (int j = lane; j < NR * NB; j += 64)
                    st_w(sadj + j, ld_w(src + j));
            } else {
                // H's rows only (sets 1 and 3 of the instance's rows); v's G
                // rows are read from HBM, one row per batch
                for (int j = lane; j < (NR / 2) * NB; j += 64)
                    st_w(sadj + j, ld_w(src + (2 * (j / NB) + 1) * NB + j % NB));
                gadj = src;
            }
            inst = i;
            map_off = (int)P.inst[i].map_off;
            nG = (int)P.inst[i].nG;
            nH = (int)P.inst[i].nH;
            target = (int)P.inst[i].target;
            inc_slot = (int)P.inst[i].inc_slot;
            twin = (int)P.inst[i].twin;
            dead_on = (int)P.inst[i].dead_on;
        }
        int g = 0;
        if (lane == 0) {
            g = ld_rlx(&P.inc[inc_slot]);
            // the twin's search already finished: nothing is left to prove
            if (twin >= 0 && ld_rlx(&P.open[twin]) == 0 && !ld_rlx(&P.dead[twin]))
                g = 255;
            // given up as a dead end
            if (dead_on && ld_rlx(&P.dead[i]))
                g = 255;
        }
        inc = cap_inc(rl(g, 0));
        sync();
    }

    __device__ void start_root(int i) {
        set_instance(i);
        DevInst di = P.inst[i];
        K = sc((int)di.K0);
        if constexpr (Q == 1) {
            if (lane < K) {
                const Cls<W> *rc = (const Cls<W> *)P.rootcls + sc((int)di.cls_off);
                scls[lane] = rc[lane];
            }
        } else {
            const Cls<W> *rc = (const Cls<W> *)P.rootcls + sc((int)di.cls_off);
            for (int j = lane; j < K; j += 64)
                st_cls(scls + j, ld_cls(rc + j));
        }
        sync();
        t = 0;
        base = 0;
        d = 0;
        d0 = 0;
        load_regs();
        int contrib = 0;
        if constexpr (Q == 1) {
            if (lane < K) {
                int nl = popc(cL), nr = popc(cR);
                contrib = nl < nr ? nl : nr;
            }
        } else {
            // (slots past K hold empty classes)
            if (lane < (1 << logS)) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int nl = popc(slotL(q)), nr = popc(slotR(q));
                    contrib += nl < nr ? nl : nr;
                }
            }
        }
        bound = wave_sum(contrib);
        c_nodes += 1;  // the root
        if (K == 0 || bound <= inc) {
            rrem = 0;
            flags = 0;
            return;
        }
        flags = kFlagUnmatched;
        select();
    }

    // -- incumbent ---------------------------------------------------------------

    __device__ void improve(int size) {
        int old = 0;
        if (lane == 0)
            old = a_max(&P.inc[inc_slot], size);
        old = rl(old, 0);
        if (old < size) {
            uint16_t *dst = P.maps + map_off + size * (size - 1) / 2;
            if constexpr (Q == 1) {
                if (lane < size)
                    dst[lane] = smap[lane];
            } else {
                for (int j = lane; j < size; j += 64)
                    dst[j] = smap[j];
            }
            if (lane == 0) {
                a_max64(&P.t_best[inst], ((unsigned long long)size << 48) |
                                             (now_ticks() & 0xFFFFFFFFFFFFull));
                // the nodes that led to this improvement (dead-end forecast)
                a_max64(&P.best_nodes[inst],
                        ld_rlx(&P.nodes[inst]) + pend_nodes + c_nodes);
            }
        }
        set_inc(old > size ? old : size);
    }

    // The local incumbent used for pruning.  Once a goal size is reached
    // (goal-directed search), it jumps above every possible bound so that
    // the rest of the instance's work prunes away at once.
    __device__ int cap_inc(int x) const { return (target > 0 && x >= target) ? 255 : x; }
    __device__ void set_inc(int x) {
        x = cap_inc(x);
        if (x > inc)
            inc = x;
    }

    // -- one batch of sibling children -----------------------------------------

    __device__ void batch() {
        if constexpr (Q > 1) {
            batch_wide();
            return;
        }
        const int S = 1 << logS;
        int C = popc(rrem);
        if (C > cmax)
            C = cmax;
        if (C > (64 >> logS))
            C = 64 >> logS;
        const int seg = lane >> logS;
        const bool act = seg < C;
        // partners in the policy's order (policy kernels only)
        const bool ordered = POL && (flags & kFlagOrdered);

        // this lane's partner w: segment seg takes the seg-th of the next C
        // partners (lowest indices first, or the policy's order)
        int myw = 0;
        int wl[8];
        if (ordered) {
            W rr = rrem;
            int pos = 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                wl[c] = 0;
                if (c < C) {
                    while (pos < 63 && !((rr >> sord[t * 64 + pos]) & 1))
                        ++pos;
                    int wc = sc((int)sord[t * 64 + pos]);
                    ++pos;
                    rr &= ~((W)1 << wc);
                    wl[c] = wc;
                }
            }
            myw = wl[0];
#pragma unroll
            for (int c = 1; c < 8; ++c)
                if (c < C)
                    myw = seg == c ? wl[c] : myw;
        } else {
            // drop the seg lowest vertices of rrem, then take the lowest
            W x = rrem;
            for (int i = 1; i < C; ++i) {
                W y = x & (x - 1);
                x = seg >= i ? y : x;
            }
            myw = act ? ctz(x) : 0;
        }
        const W vb = (W)1 << v;
        const W Lx = cL & ~vb;
        const W Rx = cR & ~((W)1 << myw);

        // filterDomain: parts by adjacency letter
        W pl[NR], pr[NR];
        const W go = sadj[v], ho = sadj[NB + myw];
        if constexpr (!DIR) {
            pl[0] = Lx & ~go;
            pr[0] = Rx & ~ho;
            pl[1] = Lx & go;
            pr[1] = Rx & ho;
        } else {
            const W gi = sadj[2 * NB + v], hi = sadj[3 * NB + myw];
            pl[0] = Lx & ~go & ~gi;
            pr[0] = Rx & ~ho & ~hi;
            pl[1] = Lx & go & ~gi;
            pr[1] = Rx & ho & ~hi;
            pl[2] = Lx & ~go & gi;
            pr[2] = Rx & ~ho & hi;
            pl[3] = Lx & go & gi;
            pr[3] = Rx & ho & hi;
        }
        int contrib = 0;
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            int nl = popc(pl[a]), nr = popc(pr[a]);
            contrib += nl < nr ? nl : nr;
        }
        if (!act)
            contrib = 0;

        // Eq. 1 per segment, decided in each segment's last lane
        const int b = d + 1 + seg_sum(contrib, logS);
        const bool rep = (lane & (S - 1)) == S - 1;
        const uint64_t sb = ballot(act && rep && b > inc);
        const int nsurv = __builtin_popcountll(sb);
        const int first = sb ? (ctz(sb) >> logS) : -1;
        const int fb = sb ? rl(b, ctz(sb)) : 0;
        c_nodes += (uint32_t)(C - nsurv + (nsurv ? 1 : 0));
        c_batches += 1;
        c_children += (uint32_t)C;
        c_lanes += (uint32_t)(C * K);
        c_ncls += (uint32_t)((C - nsurv + (nsurv ? 1 : 0)) * K);

        // drop the pruned children and the one we descend into; the other
        // survivors stay in rrem and are evaluated again after the descent
        int wF = 0;
        if (ordered) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (c < C) {
                    bool keep = ((sb >> (((c << logS) + S - 1) & 63)) & 1) && c != first;
                    if (!keep)
                        rrem &= ~((W)1 << wl[c]);
                    if (c == first)
                        wF = wl[c];
                }
            }
        } else {
            // lane j stands for vertex j; the child of rank r took the r-th
            // lowest vertex of rrem
            const bool inR = lane < NB && ((rrem >> (lane & (NB - 1))) & 1);
            const int r = mbcnt((uint64_t)rrem);
            const bool taken = inR && r < C;
            const bool surv = taken && ((sb >> (((r << logS) + S - 1) & 63)) & 1);
            rrem &= ~(W)ballot(taken && (!surv || r == first));
            if (first >= 0)
                wF = ctz((uint64_t)ballot(taken && r == first));
        }
        if (first < 0)
            return;

        // compact the surviving child's non-empty classes into a new frame
        const bool inF = seg == first;
        int pos[NR];
        bool ne[NR];
        int K2 = 0;
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            ne[a] = inF && pl[a] != 0 && pr[a] != 0;
            uint64_t m = ballot(ne[a]);
            pos[a] = K2 + mbcnt(m);
            K2 += __builtin_popcountll(m);
        }
        // (the stack holds the worst case, m(m+1)/2 classes: this capacity
        // check cannot fire)
        const int nb = base + K;
        if (nb + K2 > cap_classes) {
            fail(1);
            return;
        }
        if (nb + K2 > max_used)
            max_used = nb + K2;
        // every lane stores; lanes without a class of the child hit the trash slot
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            Cls<W> c;
            c.L = pl[a];
            c.R = pr[a];
            scls[ne[a] ? nb + pos[a] : cap_classes] = c;
        }
        smap[d] = (uint16_t)(v | (wF << 8));  // the same value from every lane
        save_top();
        sync();
        if (d + 1 > inc)
            improve(d + 1);
        if (K2 == 0)
            return;  // a leaf: nothing left to split
        c_pushed += (uint32_t)K2;
        t += 1;
        base = nb;
        K = K2;
        d += 1;
        bound = fb;
        flags = kFlagUnmatched;
        load_regs();
        select();
        (void)S;
    }

    // filterDomain on slot q of this lane: the parts of class (slot q) by
    // adjacency letter, with v and w already struck from it.
    __device__ void parts_of(int q, const W &vb, const W &wb, const W &go, const W &ho,
                             const W &gi, const W &hi, W *l, W *r) const {
        const W Lx = slotL(q) & ~vb;
        const W Rx = slotR(q) & ~wb;
        if constexpr (!DIR) {
            l[0] = Lx & ~go;
            r[0] = Rx & ~ho;
            l[1] = Lx & go;
            r[1] = Rx & ho;
        } else {
            l[0] = Lx & ~go & ~gi;
            r[0] = Rx & ~ho & ~hi;
            l[1] = Lx & go & ~gi;
            r[1] = Rx & ho & ~hi;
            l[2] = Lx & ~go & gi;
            r[2] = Rx & ~ho & hi;
            l[3] = Lx & go & gi;
            r[3] = Rx & ho & hi;
        }
    }

    // batch() for rows wider than 64 bits: the same steps, on slot q too
    // when the frame has more than 64q classes (then S = 64 and the batch
    // is one child).  Lane j stands for vertices j, 64 + j, ... when the
    // children taken are struck from the partner mask.  The surviving
    // child's parts are split again when it is pushed, rather than kept
    // from the bound pass: Q slots of parts would not fit in registers.
    __device__ void batch_wide() {
        const int S = 1 << logS;
        int C = popc(rrem);
        if (C > cmax)
            C = cmax;
        if (C > (64 >> logS))
            C = 64 >> logS;
        const int seg = lane >> logS;
        const bool act = seg < C;
        W x = rrem;
        for (int i = 1; i < C; ++i) {
            W y = x & (x - (W)1);
            x = pick(seg >= i, y, x);
        }
        const int myw = act ? ctz(x) : 0;
        const W vb = bit_at<W>(v);
        const W wb = bit_at<W>(myw);
        const W go = ld_w(gadj + v), ho = ld_w(sadj + myw);
        W gi = (W)0, hi = (W)0;
        if constexpr (DIR) {
            gi = ld_w(gadj + 2 * NB + v);
            hi = ld_w(sadj + NB + myw);
        }
        int contrib = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q > 0 && K <= 64 * q)
                break;
            W l[NR], r[NR];
            parts_of(q, vb, wb, go, ho, gi, hi, l, r);
#pragma unroll
            for (int a = 0; a < NR; ++a) {
                int nl = popc(l[a]), nr = popc(r[a]);
                contrib += nl < nr ? nl : nr;
            }
        }
        if (!act)
            contrib = 0;

        const int b = d + 1 + seg_sum(contrib, logS);
        const bool rep = (lane & (S - 1)) == S - 1;
        const uint64_t sb = ballot(act && rep && b > inc);
        const int nsurv = __builtin_popcountll(sb);
        const int first = sb ? (ctz(sb) >> logS) : -1;
        const int fb = sb ? rl(b, ctz(sb)) : 0;
        c_nodes += (uint32_t)(C - nsurv + (nsurv ? 1 : 0));
        c_batches += 1;
        c_children += (uint32_t)C;
        c_lanes += (uint32_t)(C * (K < S ? K : S));
        c_ncls += (uint32_t)((C - nsurv + (nsurv ? 1 : 0)) * K);

        // the child of rank r took the r-th lowest vertex of rrem
        uint64_t xq[Q];
        int below = 0, wF = -1;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint64_t m = word64(rrem, q);
            const int r = below + mbcnt(m);
            below += __builtin_popcountll(m);
            const bool tq = ((m >> lane) & 1) && r < C;
            const bool sq = tq && ((sb >> (((r << logS) + S - 1) & 63)) & 1);
            xq[q] = ballot(tq && (!sq || r == first));
            const uint64_t f = ballot(tq && r == first);
            if (wF < 0 && f)
                wF = 64 * q + ctz(f);
        }
        rrem &= ~from_words<W>(xq);
        if (first < 0)
            return;

        // push the surviving child: its non-empty classes, compacted in
        // slot and part order (a class past the capacity goes to the trash
        // slot, and the check below then fails the search)
        const bool inF = seg == first;
        const int nb = base + K;
        int K2 = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q > 0 && K <= 64 * q)
                break;
            W l[NR], r[NR];
            parts_of(q, vb, wb, go, ho, gi, hi, l, r);
#pragma unroll
            for (int a = 0; a < NR; ++a) {
                const bool ne = inF && l[a] != (W)0 && r[a] != (W)0;
                const uint64_t m = ballot(ne);
                const int pos = nb + K2 + mbcnt(m);
                K2 += __builtin_popcountll(m);
                Cls<W> c;
                c.L = l[a];
                c.R = r[a];
                st_cls(scls + (ne && pos < cap_classes ? pos : cap_classes), c);
            }
        }
        // (the stack holds the worst case: this capacity check cannot fire)
        if (nb + K2 > cap_classes) {
            fail(1);
            return;
        }
        if (nb + K2 > max_used)
            max_used = nb + K2;
        smap[d] = (uint16_t)(v | (wF << 8));
        save_top();
        sync();
        if (d + 1 > inc)
            improve(d + 1);
        if (K2 == 0)
            return;
        c_pushed += (uint32_t)K2;
        t += 1;
        base = nb;
        K = K2;
        d += 1;
        bound = fb;
        flags = kFlagUnmatched;
        load_regs();
        select();
    }

    // -- the "v unmatched" child, done in place on the top frame -----------------
    // Its bound follows from the parent's: only the selected class loses v.
    __device__ bool unmatched() {
        flags = 0;
        int ub = bound - (lsel <= rsel ? 1 : 0);
        c_nodes += 1;
        if (ub <= inc)
            return false;
        const W vb = bit_at<W>(v);
        if constexpr (Q > 1) {
            // class j sits in lane j mod S, slot j / S
            const int S = 1 << logS;
            if (lsel == 1) {
                // the last class moves into the selected one's place
                const int last = K - 1;
                Cls<W> c;
                c.L = slotL(last >> logS);
                c.R = slotR(last >> logS);
                st_cls(scls + ((sel != last && lane == (last & (S - 1))) ? base + sel : cap_classes), c);
                K = last;
                sync();
                bound = ub;
                if (K == 0)
                    return false;
                load_regs();
            } else {
                const int sl = sel & (S - 1);
                const int sq = sel >> logS;
                const bool mine = (lane & (S - 1)) == sl;
                cL = pick(mine && sq == 0, cL & ~vb, cL);
#pragma unroll
                for (int q = 1; q < Q; ++q)
                    cLh[q - 1] = pick(mine && sq == q, cLh[q - 1] & ~vb, cLh[q - 1]);
                st_w(&scls[lane == sl ? base + sel : cap_classes].L, slotL(sq));
                sync();
                bound = ub;
            }
        } else if (lsel == 1) {
            int last = K - 1;
            Cls<W> c;
            c.L = cL;
            c.R = cR;
            scls[(sel != last && lane == last) ? base + sel : cap_classes] = c;
            K = last;
            sync();
            bound = ub;
            if (K == 0)
                return false;
            load_regs();
        } else {
            int k = lane & ((1 << logS) - 1);
            if (k == sel)
                cL &= ~vb;
            scls[lane == sel ? base + sel : cap_classes].L = cL;
            sync();
            bound = ub;
        }
        flags = kFlagUnmatched;
        select();
        return true;
    }

    // Back to the parent frame; false when the stack is empty.
    __device__ bool pop() {
        for (;;) {
            t -= 1;
            if (t < 0)
                return false;
            read_hdr(t);
            if (reprune && bound <= inc)
                continue;
            if (rrem == 0 && !(flags & kFlagUnmatched))
                continue;
            load_regs();
            return true;
        }
    }

    // -- work sharing ------------------------------------------------------------

    // A free slot in this XCD's ring, else in the next rings; false if all
    // are full (the donation is then skipped: the work stays local).  A
    // claim lost to another producer is retried up to `tries` times per ring:
    // a donation gives up early, a child that has nowhere else to go keeps
    // trying until the rings are really full.
    __device__ bool reserve(int &ring, unsigned long long &ticket, int tries_per_ring) {
        const unsigned long long mask = (unsigned long long)P.ring_slots - 1;
        int ok = 0, rr = 0;
        unsigned long long tk = 0;
        if (lane == 0) {
            for (int k = 0; k < kRings && !ok; ++k) {
                const int r = (my_ring + k) & (kRings - 1);
                unsigned long long *sq = P.seq + (size_t)r * P.ring_slots;
                for (int tries = 0; tries < tries_per_ring; ++tries) {
                    unsigned long long tl = ld_rlx(&P.g->ring[r].tail);
                    unsigned long long s = ld_rlx(&sq[tl & mask]);
                    if (s == tl) {
                        if (cas64(&P.g->ring[r].tail, tl, tl + 1)) {
                            ok = 1;
                            rr = r;
                            tk = tl;
                            break;
                        }
                    } else if (s < tl) {
                        break;  // this ring is full
                    }
                }
            }
        }
        // No acquire here: the slot's last reader had all its loads of the
        // slot returned (s_waitcnt) before it stored the sequence number we
        // read, so none of our writes below can reach them.
        ok = rl(ok, 0);
        ring = rl(rr, 0);
        ticket = rl_ull(tk, 0);
        return ok != 0;
    }

    // Give the shallowest open frame's remaining children to the queue.
    __device__ void donate() {
        int b = -1;
        W grr = 0;
        int gfl = 0;
        for (int i = 0; i < t; ++i) {
            W r = hdr_rrem(i);
            int f = hdr(i, kHFlags);
            if (hdr(i, kHD) > P.donate_depth)
                return;  // deeper frames hold too little work to hand out
            if (r != 0 || (f & kFlagUnmatched)) {
                b = i;
                grr = r;
                gfl = f & (kFlagUnmatched | kFlagOrdered);
                break;
            }
        }
        W keep_r = 0;
        if (b < 0) {
            if (d > P.donate_depth)
                return;
            int n = popc(rrem);
            if (n >= 2) {
                W r = rrem, kept = 0;
                for (int c = 0; c < n - n / 2; ++c) {
                    kept |= r & (~r + 1);
                    r &= r - 1;
                }
                grr = r;
                gfl = flags & (kFlagUnmatched | kFlagOrdered);
                keep_r = kept;
            } else if (n == 1 && (flags & kFlagUnmatched)) {
                grr = 0;
                gfl = kFlagUnmatched | (flags & kFlagOrdered);
                keep_r = rrem;
            } else {
                return;
            }
            b = t;
        }
        unsigned long long ticket;
        int ring;
        if (!reserve(ring, ticket, 4))
            return;
        const unsigned long long mask = (unsigned long long)P.ring_slots - 1;
        const size_t idx = (size_t)ring * P.ring_slots + (size_t)(ticket & mask);
        uint8_t *slot = P.slots + idx * (size_t)P.slot_bytes;
        int fK, fd, fbase;
        RecHdr<W> rh;
        if (b == t) {
            fK = K;
            fd = d;
            fbase = base;
            rh.v = (uint8_t)v;
            rh.sel = (uint8_t)sel;
            rh.bound = (uint8_t)bound;
            rh.lsel = (uint8_t)lsel;
            rh.rsel = (uint8_t)rsel;
        } else {
            fK = hdr(b, kHK);
            fd = hdr(b, kHD);
            fbase = hdr(b, kHBase);
            rh.v = (uint8_t)hdr(b, kHV);
            rh.sel = (uint8_t)hdr(b, kHSel);
            rh.bound = (uint8_t)hdr(b, kHBound);
            rh.lsel = (uint8_t)hdr(b, kHLsel);
            rh.rsel = (uint8_t)hdr(b, kHRsel);
        }
        rh.inst = (uint32_t)inst;
        rh.K = (uint8_t)fK;
        rh.d = (uint8_t)fd;
        rh.flags = (uint8_t)gfl;
        rh.pad[0] = rh.pad[1] = rh.pad[2] = rh.pad[3] = 0;
        rh.rrem = grr;
        if (lane == 0)
            *(RecHdr<W> *)slot = rh;
        uint16_t *rmap = (uint16_t *)(slot + rec_map_off<W>());
        Cls<W> *rcls = (Cls<W> *)(slot + rec_cls_off<W>());
        if constexpr (Q == 1) {
            if (lane < fd)
                rmap[lane] = smap[lane];
            if (lane < fK)
                rcls[lane] = scls[fbase + lane];
        } else {
            for (int j = lane; j < fd; j += 64)
                rmap[j] = smap[j];
            for (int j = lane; j < fK; j += 64)
                st_cls(rcls + j, ld_cls(scls + fbase + j));
        }
        if (lane == 0) {
            a_add_rlx(&P.open[inst], 1);
            a_add_rlx(&P.g->open_total, 1);
            st_rel(&P.seq[idx], ticket + 1);
        }
        if (b == t) {
            rrem = keep_r;
            flags &= kFlagOrdered;
        } else if (lane == 0) {
            shdr[b * HW + kHRremLo] = 0;
            shdr[b * HW + kHRremHi] = 0;
            shdr[b * HW + kHFlags] = 0;
#pragma unroll
            for (int k = 2; k < (int)sizeof(W) / 4; ++k)
                shdr[b * HW + rrem_field(k)] = 0;
        }
        sync();
        n_don += 1;
    }

    // Take a queued node: from this XCD's ring, else (steal) from one other
    // ring, a different one on each call.
    __device__ bool take_record() {
        const unsigned long long mask = (unsigned long long)P.ring_slots - 1;
        int ok = 0, rr = 0;
        unsigned long long hd = 0;
        if (lane == 0) {
            steal_from = (steal_from + 1) & (kRings - 1);
            if (steal_from == my_ring)
                steal_from = (steal_from + 1) & (kRings - 1);
            for (int k = 0; k < 2 && !ok; ++k) {
                const int r = k == 0 ? my_ring : steal_from;
                unsigned long long *sq = P.seq + (size_t)r * P.ring_slots;
                for (int tries = 0; tries < 4; ++tries) {
                    unsigned long long h = ld_rlx(&P.g->ring[r].head);
                    unsigned long long s = ld_rlx(&sq[h & mask]);
                    if (s == h + 1) {
                        if (cas64(&P.g->ring[r].head, h, h + 1)) {
                            ok = 1;
                            rr = r;
                            hd = h;
                            break;
                        }
                    } else if (s < h + 1) {
                        break;  // empty, or its producer is still writing
                    }
                }
            }
        }
        ok = rl(ok, 0);
        if (!ok)
            return false;
        // pairs with the producer's release store of the slot's sequence number
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        hd = rl_ull(hd, 0);
        const int ring = rl(rr, 0);
        const size_t idx = (size_t)ring * P.ring_slots + (size_t)(hd & mask);
        const uint8_t *slot = P.slots + idx * (size_t)P.slot_bytes;
        RecHdr<W> rh = *(const RecHdr<W> *)slot;
        int ri = sc((int)rh.inst);
        K = sc((int)rh.K);
        d = sc((int)rh.d);
        v = sc((int)rh.v);
        sel = sc((int)rh.sel);
        bound = sc((int)rh.bound);
        flags = sc((int)rh.flags);
        lsel = sc((int)rh.lsel);
        rsel = sc((int)rh.rsel);
        rrem = sc((W)rh.rrem);
        const uint16_t *rmap = (const uint16_t *)(slot + rec_map_off<W>());
        const Cls<W> *rcls = (const Cls<W> *)(slot + rec_cls_off<W>());
        // entry lane + 64q of the mapping and of the classes in slot q
        uint16_t mp[Q];
        Cls<W> cc[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            mp[q] = 0;
            cc[q].L = (W)0;
            cc[q].R = (W)0;
            if (lane + 64 * q < d)
                mp[q] = rmap[lane + 64 * q];
            if (lane + 64 * q < K)
                cc[q] = ld_cls(rcls + lane + 64 * q);
        }
        // every lane's loads of the slot have returned before the slot is
        // handed back, so a relaxed store suffices: the producer's later
        // writes cannot reach values already in registers (the signal fence
        // keeps the compiler from moving the store above the loads)
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0)
            st_rlx(&P.seq[idx], hd + (unsigned long long)P.ring_slots);
        set_instance(ri);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (lane + 64 * q < d)
                smap[lane + 64 * q] = mp[q];
            if (lane + 64 * q < K)
                st_cls(scls + lane + 64 * q, cc[q]);
        }
        sync();
        t = 0;
        base = 0;
        d0 = d;
        load_regs();
        if (bound <= inc) {
            rrem = 0;
            flags = 0;
        } else if (flags & kFlagFresh) {
            flags = kFlagUnmatched;
            select();
        } else if (POL && (flags & kFlagOrdered)) {
            if constexpr (POL)
                order_partners(rrem);
        } else {
            flags &= ~kFlagOrdered;
        }
        n_pops += 1;
        return true;
    }

    // Take the next unclaimed instance.  Its work unit was counted in
    // open_total and open[i] by the reset, so nothing is added here.
    __device__ bool claim_instance() {
        if (!roots_left)
            return false;
        int i = -1;
        if (lane == 0) {
            unsigned nx = ld_rlx(&P.g->next_inst);
            if (nx < (unsigned)P.count) {
                unsigned x = a_addu(&P.g->next_inst, 1u);
                if (x < (unsigned)P.count)
                    i = (int)x;
            }
        }
        i = rl(i, 0);
        if (i < 0) {
            roots_left = false;
            return false;
        }
        start_root(i);
        return true;
    }

    __device__ void fold() {
        pend_nodes += c_nodes;
        n_batches += c_batches;
        n_children += c_children;
        n_lanes += c_lanes;
        n_pushed += c_pushed;
        n_ncls += c_ncls;
        c_nodes = c_batches = c_children = c_lanes = c_pushed = c_ncls = 0;
    }

    __device__ void flush_nodes() {
        fold();
        if (pend_nodes && inst >= 0 && lane == 0) {
            a_add64(&P.nodes[inst], pend_nodes);
            if (P.node_limit > 0) {
                unsigned long long tot = a_add64(&P.g->node_total, pend_nodes) + pend_nodes;
                if ((long long)tot > P.node_limit)
                    raise_flag(kFlagStop);
            }
        }
        pend_nodes = 0;
    }

    // Periodic: refresh the incumbent, honour limits, keep the queue
    // stocked.  Every line read here is per instance or per XCD: a check
    // never touches a line that all wavefronts of the chip update.
    __device__ void check() {
        since_check = 0;
        fold();
        // the queue is read only when some frame of this unit may be donated
        const bool may_donate = !P.single_wave && P.donate_low >= 0 && d0 <= P.donate_depth;
        unsigned long long hd = 0, tl = 0;
        int gi = 0;
        unsigned fl = 0;
        if (lane == 0) {
            gi = ld_rlx(&P.inc[inc_slot]);
            if (twin >= 0 && ld_rlx(&P.open[twin]) == 0 && !ld_rlx(&P.dead[twin]))
                gi = 255;
            if (dead_on && ld_rlx(&P.dead[inst]))
                gi = 255;
            fl = ld_rlx(&P.g->xcd[my_ring].flag);
            if (may_donate) {
                tl = ld_rlx(&P.g->ring[my_ring].tail);
                hd = ld_rlx(&P.g->ring[my_ring].head);
            }
        }
        gi = rl(gi, 0);
        if (gi > inc)
            set_inc(gi);
        // (the done flag cannot be up while this unit is alive: a set flag
        // is a stop)
        if (rl(fl, 0)) {
            stop = true;
            return;
        }
        if (now_ticks() - t_start > P.limit_ticks) {
            raise_flag(kFlagStop);
            stop = true;
            return;
        }
        if (P.node_limit > 0 || P.dead_abs > 0)
            flush_nodes();
        if (P.dead_abs > 0 && dead_on) {
            // dead-end forecast (paper Sec. IV.A): more than dead_abs nodes
            // -- and, with dead_rel, more than dead_rel times the nodes that
            // led to the last improvement -- without raising the incumbent
            int gave_up = 0;
            if (lane == 0) {
                const unsigned long long n = ld_rlx(&P.nodes[inst]);
                const unsigned long long b = ld_rlx(&P.best_nodes[inst]);
                const unsigned long long since = n > b ? n - b : 0ull;
                unsigned long long thr = (unsigned long long)P.dead_abs;
                if (P.dead_rel > 0 && (unsigned long long)P.dead_rel * b > thr)
                    thr = (unsigned long long)P.dead_rel * b;
                if (since > thr) {
                    st_rlx(&P.dead[inst], 1);
                    gave_up = 1;
                }
            }
            if (rl(gave_up, 0))
                set_inc(255);
        }
        if (may_donate) {
            // keep at least donate_low records waiting in this XCD's ring
            long long waiting = (long long)(rl_ull(tl, 0) - rl_ull(hd, 0));
            if (waiting < P.donate_low)
                donate();
        }
    }

    // The frame state is the same in every lane; saying so lets the
    // compiler keep it in scalar registers and the per-child bookkeeping on
    // the scalar unit (its divergence analysis cannot see through the loop).
    __device__ void uniformize() {
        t = sc(t);
        base = sc(base);
        K = sc(K);
        d = sc(d);
        v = sc(v);
        sel = sc(sel);
        bound = sc(bound);
        flags = sc(flags);
        lsel = sc(lsel);
        rsel = sc(rsel);
        rrem = sc(rrem);
        logS = sc(logS);
        inc = sc(inc);
        since_check = sc(since_check);
    }

    // Depth-first search from the frame loaded at level 0.
    __device__ void run() {
        while (!stop) {
            uniformize();
            if (rrem != 0) {
                batch();
            } else if (flags & kFlagUnmatched) {
                if (!unmatched() && !pop())
                    break;
            } else if (!pop()) {
                break;
            }
            if (++since_check >= check_interval)
                check();
        }
    }

    __device__ void finish_unit() {
        flush_nodes();
        if (!stop && lane == 0) {
            int r = a_add_rlx(&P.open[inst], -1);
            if (r == 1)
                __hip_atomic_store(&P.t_proof[inst], now_ticks(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            // a unit is only made by a live unit, so the count reaches zero
            // once, when the last one ends: that wavefront says so to all
            if (a_add_rlx(&P.g->open_total, -1) == 1)
                raise_flag(kFlagDone);
        }
    }

    __device__ void main_loop() {
        t_start = now_ticks();
        if (lane == 0)
            a_min64(&P.g->t0, t_start);
        int backoff = 0;
        for (;;) {
            bool got = false;
            if (!P.single_wave)
                got = take_record();
            if (!got)
                got = claim_instance();
            if (got) {
                backoff = 0;
                const unsigned long long t_unit = now_ticks();
                run();
                finish_unit();
                n_busy += now_ticks() - t_unit;
                if (stop)
                    break;
                continue;
            }
            unsigned fl = 0;
            if (lane == 0)
                fl = ld_rlx(&P.g->xcd[my_ring].flag);
            if (rl(fl, 0))
                break;  // stopped, or no work is left anywhere
            if (now_ticks() - t_start > P.limit_ticks) {
                raise_flag(kFlagStop);
                break;
            }
            // back off: 1, 2, 4, ... backoff_max sleeps of about 8k cycles
            // (3.4 us).  Polling more often slows the busy wavefronts more
            // than it feeds the idle ones: the polls contend with their
            // checks on the same ring lines.
            const int bmax = P.backoff_max;
            backoff = backoff ? (2 * backoff < bmax ? 2 * backoff : bmax) : 1;
            const unsigned long long t_sleep = now_ticks();
            for (int i = 0; i < backoff; ++i)
                __builtin_amdgcn_s_sleep(127);
            n_sleep += now_ticks() - t_sleep;
        }
        fold();
        if (lane == 0) {
            a_add64(&P.g->batches, n_batches);
            a_add64(&P.g->children, n_children);
            a_add64(&P.g->lane_slots, n_lanes);
            a_add64(&P.g->donations, n_don);
            a_add64(&P.g->pops, n_pops);
            a_add64(&P.g->busy_ticks, n_busy);
            a_add64(&P.g->pushed_classes, n_pushed);
            a_add64(&P.g->node_classes, n_ncls);
            a_add64(&P.g->sleep_ticks, n_sleep);
            __hip_atomic_fetch_max(&P.g->max_stack, max_used, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
};

template <typename W, bool DIR, bool POL>
__global__ void __launch_bounds__(256) mcs_search_kernel(SearchParams Pk) {
    extern __shared__ __align__(16) uint8_t smem[];
    // The parameters live in LDS, not in scalar registers for the whole
    // kernel: the search loop needs few of them, and scalar registers are
    // what its state lives in.
    __shared__ SearchParams P;
    if (threadIdx.x == 0)
        P = Pk;
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    if (Pk.single_wave && (blockIdx.x != 0 || wv != 0))
        return;
    Searcher<W, DIR, POL> s(P, smem + (size_t)wv * (size_t)Pk.lds_per_wave,
                            (int)(blockIdx.x * (blockDim.x >> 6)) + wv);
    s.main_loop();
}

// Clears the per-run state with plain stores (no memset nodes, so the pair
// of kernels can be replayed from a HIP graph).
__global__ void __launch_bounds__(256) mcs_reset_kernel(ResetParams R) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    for (int i = tid; i < R.count; i += stride) {
        R.inc[i] = R.inst[i].lb;
        R.open[i] = 1;  // the unclaimed root
        R.nodes[i] = 0;
        R.t_best[i] = 0;
        R.t_proof[i] = 0;
        R.best_nodes[i] = 0;
        R.dead[i] = 0;
    }
    for (int i = tid; i < kRings * R.ring_slots; i += stride)
        R.seq[i] = (unsigned long long)(i % R.ring_slots);
    if (tid == 0) {
        DevGlobals z = {};
        z.t0 = ~0ull;
        z.open_total = R.count;
        if (R.count == 0)
            for (int k = 0; k < kRings; ++k)
                z.xcd[k].flag = kFlagDone;
        *R.g = z;
    }
}

}  // namespace mcs

// ---- launch entry points used by the host driver ---------------------------

extern "C" void *mcs_internal_search_kernel(int word_bytes, int directed, int policy) {
    using namespace mcs;
    if (word_bytes == 16 || word_bytes == 32) {
        // (the learned policy takes graphs of at most 64 vertices)
        if (policy)
            return nullptr;
        if (word_bytes == 32)
            return directed ? (void *)mcs_search_kernel<u256, true, false>
                            : (void *)mcs_search_kernel<u256, false, false>;
        return directed ? (void *)mcs_search_kernel<u128, true, false>
                        : (void *)mcs_search_kernel<u128, false, false>;
    }
    if (word_bytes == 4) {
        if (policy)
            return directed ? (void *)mcs_search_kernel<uint32_t, true, true>
                            : (void *)mcs_search_kernel<uint32_t, false, true>;
        return directed ? (void *)mcs_search_kernel<uint32_t, true, false>
                        : (void *)mcs_search_kernel<uint32_t, false, false>;
    }
    if (policy)
        return directed ? (void *)mcs_search_kernel<uint64_t, true, true>
                        : (void *)mcs_search_kernel<uint64_t, false, true>;
    return directed ? (void *)mcs_search_kernel<uint64_t, true, false>
                    : (void *)mcs_search_kernel<uint64_t, false, false>;
}

extern "C" void *mcs_internal_reset_kernel(void) { return (void *)mcs::mcs_reset_kernel; }
