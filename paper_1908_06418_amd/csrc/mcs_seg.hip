// McSplit search with one depth-first search per lane segment (gfx950).
//
// The work per search node is the paper's Solve body (Sec. II.B, Algorithm 1):
// split every label class by adjacency to v (G side) and to w (H side) --
// filterDomain -- and bound the child with Eq. 1,
//     bound = |M| + sum over classes of min(|L|, |R|),
// pruning it when the bound cannot beat the incumbent.
//
// Layout (ours): a wavefront is cut into 64 / S segments of S = 4, 8 or 16
// lanes, and each segment runs its own search.  Lane k of a segment holds
// class k of the segment's top frame (classes k + S, k + 2S, ... of a frame
// with more than S classes are read from LDS in further passes).  Every
// per-search value -- the frame (depth, selected class, v, remaining
// partners, bound), the instance, the incumbent -- is a vector register that
// is uniform within the segment, so the search's bookkeeping runs on the
// vector unit for all segments at once instead of on the CU's single scalar
// unit.  Segment reductions (the Eq. 1 sum, the class-choice minimum) are
// DPP steps that stay inside 4-, 8- or 16-lane groups.
//
// The segments advance in lock step.  One step is, for each segment, in this
// order and only where it applies:
//   pop       -- the top frame has nothing left: return to the parent frame;
//   unmatched -- the top frame's partners are done: take its "v unmatched"
//                child in place (its bound follows from the parent's);
//   reload    -- a frame the search has just entered, or returned to, gets
//                its classes into registers and, if it is new, its class
//                and v chosen;
//   evaluate  -- split the classes for the next partner w of v, bound the
//                child, and either prune it or push it as the new top frame
//                (to be reloaded at the next step).
// A phase no segment needs is skipped (a uniform branch on a ballot), and
// each phase's code runs at most once per step for all the segments that
// need it.  Children are evaluated one per step, in ascending w, each
// exactly once.
//
// Work sharing, incumbents and termination are those of the one-search-per-
// wavefront kernel (mcs_search.hip), applied per segment: node records in
// per-XCD rings in HBM (a segment with no work takes one, or claims the next
// unstarted instance), a busy segment donates its shallowest open frame when
// its XCD's ring runs low, per-instance incumbents raised by atomicMax, and a
// count of live work units whose last decrement raises the done flag.
#include "mcs_device.h"

namespace mcs {

// Frame header of a segment: two 32-bit words (one 8-byte LDS access).
//   x: base (first class, 12 bits) | K << 12 | d << 19 | v << 26
//   y: sel | bound << 6 | unmatched << 13 | lo << 14
// The remaining partners of v are not stored as a mask: partners are taken
// in ascending order and a donation from the top frame hands out the lower
// part of the rest, so they are always the selected class's R_sel above one
// vertex -- lo, the partner taken last, plus one (kNoPartners: none left) --
// and, in a unit's bottom frame only, at most hi0 (a register: the unit may
// have come from a record holding a lower part).  The mask is rebuilt from
// R_sel when the search returns to the frame.  |L_sel| and |R_sel| are not
// stored either: the selected class itself is not changed while its frame
// is open (only its partner copy is), so they are counted from it when they
// are needed.
constexpr uint32_t kNoPartners = 127;

// Codes of DevGlobals::error (the host reports MCS_E_INTERNAL).
constexpr unsigned kErrMapping = 2;  // a mapping larger than the smaller graph
constexpr unsigned kErrStack = 3;    // a frame past the class stack's worst case

// Flags of a segment's top frame beside kFlagUnmatched, set between phases
// of a step (never stored in a frame header or record):
constexpr int kFlagSelect = 4;  // a new frame: load its classes, choose class and v
constexpr int kFlagLoad = 8;    // a frame returned to: load its classes
static_assert(kFlagSelect == kFlagFresh, "a fresh record takes the same path");

// One step of a segment minimum.  The neighbour's value comes with the
// minimum's identity as the fallback, so the DPP move folds into the
// v_min_u32 itself (one instruction per step).
template <int CTRL>
DEV uint32_t dpp_min_step(uint32_t x) {
    return umin(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, CTRL, 0xF, 0xF,
                                                         false));
}

// Pointers typed by address space.  The class stack's LDS part and HBM part
// are reached through them, so the compiler emits LDS (ds_*) and global
// accesses and cannot fold the branch between the two parts into a single
// flat access with a selected address.
template <typename T>
using lds_p = __attribute__((address_space(3))) T *;
template <typename T>
using glb_p = __attribute__((address_space(1))) T *;

template <typename W, bool DIR, int LOGS>
struct SegSearch {
    static constexpr int S = 1 << LOGS;    // lanes per segment
    static constexpr int NSEG = 64 / S;    // searches per wavefront
    static constexpr int NB = bits_of<W>();
    static constexpr int NR = DIR ? 4 : 2;
    static constexpr uint32_t SEGMASK = S == 32 ? 0xFFFFFFFFu : ((1u << S) - 1);
    // lane 0 of every segment
    static constexpr uint64_t kLeadLanes = S == 16 ? 0x0001000100010001ull
                                          : S == 8 ? 0x0101010101010101ull
                                                   : 0x1111111111111111ull;

    const SearchParams &P;
    // knobs (wave-uniform)
    int cap, check_interval, reprune, arows;
    // lane identity
    int lane, lk, seg;
    // this lane's segment's LDS
    // class stack entry i is the pair of words (L, R) at 2i, 2i + 1
    lds_p<W> scls;    // [cap]: entries 0 .. cap - 1
    glb_p<W> hcls;    // entries cap and above, in HBM (the worst case fits:
                      // frames never straddle the two parts)
    glb_p<W> hwave;   // the wavefront's HBM class stacks (segment j at j * hstride)
    long long hstride;  // classes per segment's HBM part
    W *sadj;          // [NR / 2][arows] H rows: out (and in, directed)
    const W *gadj;    // all instances' rows in HBM ([count][NR][NB]: G out, H out, G in, H in)
    uint16_t *smap;   // [frames] g | h << 8 per depth
    uint2 *shdr;      // [frames]
    uint8_t *wlds;    // the wavefront's LDS (segment j at j * seg_bytes)
    int seg_bytes;

    // ---- per-segment state (uniform within a segment) ----
    int inst;         // instance of the segment's unit, -1: no unit
    int adj_inst;     // instance whose rows are in the segment's LDS
    int inc_slot, twin, map_off, target;
    int dead_on;      // the instance may be given up as a dead end
    int t, base, K, d, v, sel, bound, flags, inc, d0;
    int hi0;          // partners of the unit's bottom frame are below this vertex
    W rrem;
    W cL, cR;         // this lane's class of the top frame (class lk)
    W go, gi;         // G's out-row (and in-row) of the top frame's v
    uint32_t nodes_pend;  // nodes of the unit not yet added to the instance's count
    bool fin;         // the unit is finished (its stack emptied)
    unsigned long long pushed;  // classes in the frames this segment pushed

    // ---- wave-level ----
    bool stop;
    bool roots_left;
    int my_ring, steal_from;
    int since_check;
    int donor;        // segment considered first for the next donation
    unsigned long long t_start;
    unsigned long long n_steps, n_evals, n_nodes_wave, n_lanes, n_don, n_pops, n_busy, n_hbm,
        n_sleep, n_pushed;
    unsigned long long n_ncls;  // classes of this segment's evaluated children past the
                                // first pass (summed over the segments at the end)
    int max_used;

    __device__ SegSearch(const SearchParams &p, uint8_t *wave_lds, long long wave) : P(p) {
        lane = lane_id();
        lk = lane & (S - 1);
        seg = lane >> LOGS;
        cap = sc(p.cap_classes);
        check_interval = sc(p.check_interval);
        reprune = sc(p.reprune);
        arows = sc(p.arows);
        seg_bytes = sc(p.seg_bytes);
        wlds = wave_lds;
        const SegLayout L = seg_layout((int)sizeof(W), DIR ? 1 : 0, p.cap_classes, p.arows,
                                       p.frames);
        uint8_t *mine = wave_lds + (size_t)seg * (size_t)seg_bytes;
        scls = (lds_p<W>)(mine + L.cls);
        hstride = p.hstack_stride / (long long)sizeof(Cls<W>);
        hwave = (glb_p<W>)p.hstack + 2 * wave * NSEG * hstride;
        hcls = hwave + 2 * seg * hstride;
        sadj = (W *)(mine + L.adj);
        gadj = (const W *)p.adj;
        smap = (uint16_t *)(mine + L.map);
        shdr = (uint2 *)(mine + L.hdr);
        inst = -1;
        adj_inst = -1;
        inc_slot = 0;
        twin = -1;
        map_off = 0;
        target = 0;
        dead_on = 0;
        t = -1;
        base = K = d = v = sel = bound = flags = inc = d0 = 0;
        hi0 = NB;
        rrem = cL = cR = go = gi = 0;
        nodes_pend = 0;
        fin = false;
        pushed = 0;
        stop = false;
        roots_left = true;
        my_ring = (int)(blockIdx.x & (kRings - 1));
        steal_from = my_ring;
        since_check = 0;
        donor = 0;
        n_steps = n_evals = n_nodes_wave = n_lanes = n_don = n_pops = n_busy = n_hbm = 0;
        n_sleep = n_pushed = n_ncls = 0;
        max_used = 0;
    }

    // ---- segment helpers ----

    // Sum over the segment, in every lane of it.
    __device__ int ssum(int x) const {
        x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
        x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
        if (LOGS >= 3)
            x += dpp<0x141>(x);  // row_half_mirror: the other quad of the 8-lane half
        if (LOGS >= 4)
            x += dpp<0x140>(x);  // row_mirror: the other half of the 16-lane row
        return x;
    }
    // Minimum over the segment, in every lane of it.
    __device__ uint32_t smin(uint32_t x) const {
        x = dpp_min_step<0xB1>(x);
        x = dpp_min_step<0x4E>(x);
        if (LOGS >= 3)
            x = dpp_min_step<0x141>(x);
        if (LOGS >= 4)
            x = dpp_min_step<0x140>(x);
        return x;
    }
    // Lane 0 of the segment's value, in every lane of it.
    __device__ int sfirst(int x) const {
        return __builtin_amdgcn_ds_bpermute((lane & ~(S - 1)) << 2, x);
    }
    // This segment's bits of a ballot.
    __device__ uint32_t sbits(uint64_t m) const { return (uint32_t)(m >> (seg << LOGS)) & SEGMASK; }
    __device__ int below(uint32_t bits) const {
        return __builtin_popcount(bits & ((1u << lk) - 1u));
    }
    // Segment j's value of a per-segment register, as a scalar.
    DEV int of(int x, int j) { return rl(x, j << LOGS); }
    DEV W ofw(W x, int j) { return (W)rl((uint64_t)x, j << LOGS); }

    // Segment j's LDS.
    __device__ Cls<W> *cls_of(int j) const {
        const SegLayout L = seg_layout((int)sizeof(W), DIR ? 1 : 0, P.cap_classes, arows, P.frames);
        return (Cls<W> *)(wlds + (size_t)j * seg_bytes + L.cls);
    }
    // Class stack entry i of this lane's segment (LDS below cap, HBM above).
    __device__ Cls<W> cget(int i) const {
        Cls<W> c;
        if (i < cap) {
            c.L = scls[2 * i];
            c.R = scls[2 * i + 1];
        } else {
            c.L = hcls[2 * (i - cap)];
            c.R = hcls[2 * (i - cap) + 1];
        }
        return c;
    }
    __device__ void cput(int i, const Cls<W> &c) const {
        if (i < cap) {
            scls[2 * i] = c.L;
            scls[2 * i + 1] = c.R;
        } else {
            hcls[2 * (i - cap)] = c.L;
            hcls[2 * (i - cap) + 1] = c.R;
        }
    }
    // Entry i of segment j's class stack.
    __device__ Cls<W> cget_of(int j, int i) const {
        if (i < cap)
            return cls_of(j)[i];
        const glb_p<W> h = hwave + 2 * ((long long)j * hstride + (i - cap));
        Cls<W> c;
        c.L = h[0];
        c.R = h[1];
        return c;
    }
    // Orders a segment's class stores before other lanes of the wavefront
    // read them: an LDS frame needs only the wave's in-order LDS; a frame in
    // HBM needs its stores completed first.
    __device__ void sync_frame(bool in_hbm) const {
        if (ballot(in_hbm))
            wave_sync_global();
        else
            wave_sync();
    }

    __device__ W *adj_of(int j) const {
        const SegLayout L = seg_layout((int)sizeof(W), DIR ? 1 : 0, P.cap_classes, arows, P.frames);
        return (W *)(wlds + (size_t)j * seg_bytes + L.adj);
    }
    __device__ uint16_t *map_of(int j) const {
        const SegLayout L = seg_layout((int)sizeof(W), DIR ? 1 : 0, P.cap_classes, arows, P.frames);
        return (uint16_t *)(wlds + (size_t)j * seg_bytes + L.map);
    }
    __device__ uint2 *hdr_of(int j) const {
        const SegLayout L = seg_layout((int)sizeof(W), DIR ? 1 : 0, P.cap_classes, arows, P.frames);
        return (uint2 *)(wlds + (size_t)j * seg_bytes + L.hdr);
    }

    // ---- frames ----

    // The header of the top frame, whose partner w has just been taken.
    __device__ void save_hdr(int w) {
        uint2 h;
        h.x = (uint32_t)base | ((uint32_t)K << 12) | ((uint32_t)d << 19) | ((uint32_t)v << 26);
        h.y = (uint32_t)sel | ((uint32_t)bound << 6) |
              ((uint32_t)(flags & kFlagUnmatched) << 13) | ((uint32_t)(w + 1) << 14);
        if (lk == 0)
            shdr[t] = h;
    }
    // The partners of R above lo (the last partner taken, plus one) and
    // below hi.
    DEV W partner_range(W R, uint32_t lo1, int hi) {
        if (lo1 >= (uint32_t)NB)
            return (W)0;
        W r = R & ~(((W)1 << lo1) - 1);
        if (hi < NB)
            r &= ((W)1 << hi) - 1;
        return r;
    }
    // Header fields of frame i; the remaining partners are rebuilt from
    // R_sel, which stays in the class stack while the frame is open.
    __device__ void read_hdr(int i) {
        const uint2 h = shdr[i];
        base = (int)(h.x & 0xFFFu);
        K = (int)((h.x >> 12) & 0x7Fu);
        d = (int)((h.x >> 19) & 0x7Fu);
        v = (int)(h.x >> 26);
        sel = (int)(h.y & 0x3Fu);
        bound = (int)((h.y >> 6) & 0x7Fu);
        flags = (int)((h.y >> 13) & 1u);
        const uint32_t lo1 = (h.y >> 14) & 0x7Fu;
        rrem = lo1 < (uint32_t)NB ? partner_range(cget(base + sel).R, lo1, i == 0 ? hi0 : NB)
                                  : (W)0;
    }

    // Class lk of the top frame into registers.
    __device__ void load_regs() {
        const bool in = lk < K;
        const Cls<W> c = cget(base + (in ? lk : 0));
        cL = in ? c.L : (W)0;
        cR = in ? c.R : (W)0;
    }

    // selectLabelClass + selectVertex: the class of smallest max(|L|, |R|),
    // ties to the one holding the smallest G vertex; v = that vertex.  The
    // key carries the class index in its low byte (never deciding: L sets
    // are disjoint, so ctz(L) already differs between classes).
    __device__ void select() {
        uint32_t key = 0xFFFFFFFFu;
        if (lk < K) {
            const int nl = popc(cL), nr = popc(cR);
            key = ((uint32_t)(nl > nr ? nl : nr) << 16) | ((uint32_t)ctz(cL) << 8) | (uint32_t)lk;
        }
        if (ballot(K > S) != 0) {  // (rare) classes past the first S
            for (int c = 1; ballot(c * S < K) != 0; ++c) {
                const int k = c * S + lk;
                if (k < K) {
                    const Cls<W> x = cget(base + k);
                    const int nl = popc(x.L), nr = popc(x.R);
                    key = umin(key, ((uint32_t)(nl > nr ? nl : nr) << 16) |
                                        ((uint32_t)ctz(x.L) << 8) | (uint32_t)k);
                }
            }
        }
        const uint32_t mk = smin(key);
        v = (int)((mk >> 8) & 0xFFu);
        sel = (int)(mk & 0xFFu);
        rrem = cget(base + sel).R;
        flags = kFlagUnmatched;
        if (t == 0)
            hi0 = NB;  // a unit's bottom frame with a new class: all of its partners
    }

    // ---- incumbent ----

    __device__ int cap_inc(int x) const { return (target > 0 && x >= target) ? 255 : x; }
    __device__ void set_inc(int x) {
        x = cap_inc(x);
        inc = x > inc ? x : inc;
    }

    // The path smap[0 .. size-1] is a common induced subgraph of `size`
    // vertices: raise the instance's incumbent; the segment that raised it
    // to `size` writes the mapping into that size's slot.
    __device__ void improve(int size) {
        // a mapping larger than the smaller graph can only come from a broken
        // class partition: stop with an internal error instead of writing
        // past this instance's mapping slots
        const DevInst di = P.inst[inst];
        if (size > (di.nG < di.nH ? (int)di.nG : (int)di.nH)) {
            if (lk == 0)
                fail_lane(kErrMapping);
            return;
        }
        int old = 0;
        if (lk == 0)
            old = a_max(&P.inc[inc_slot], size);
        old = sfirst(old);
        if (old < size) {
            uint16_t *dst = P.maps + map_off + size * (size - 1) / 2;
            for (int j = lk; j < size; j += S)
                dst[j] = smap[j];
            if (lk == 0) {
                a_max64(&P.t_best[inst], ((unsigned long long)size << 48) |
                                             (now_ticks() & 0xFFFFFFFFFFFFull));
                // the nodes that led to this improvement (for the dead-end
                // forecast)
                a_max64(&P.best_nodes[inst], ld_rlx(&P.nodes[inst]) + nodes_pend);
            }
        }
        set_inc(old > size ? old : size);
    }

    // ---- the three phases of a step ----

    __device__ void pop() {
        t -= 1;
        if (t < 0) {
            fin = true;
            rrem = 0;
            flags = 0;
            return;
        }
        read_hdr(t);
        if (reprune && bound <= inc) {
            rrem = 0;
            flags = 0;  // nothing here can beat the incumbent: pop again
            return;
        }
        if (rrem != 0)
            flags |= kFlagLoad;  // its next partner is evaluated in this step
    }

    // The "v unmatched" child, in place: only the selected class loses v.
    __device__ void unmatched() {
        flags = 0;
        const Cls<W> cs = cget(base + sel);
        const int lsel = popc(cs.L), rsel = popc(cs.R);
        const int ub = bound - (lsel <= rsel ? 1 : 0);
        nodes_pend += 1;
        if (ub <= inc)
            return;
        const W vb = (W)1 << v;
        if (lsel == 1) {
            // the class empties on the G side: the last class takes its place
            const int last = K - 1;
            if (sel != last) {
                const Cls<W> c = cget(base + last);
                if (lk == 0)
                    cput(base + sel, c);
            }
            K = last;
        } else {
            Cls<W> c = cs;
            c.L &= ~vb;
            if (lk == 0)
                cput(base + sel, c);
        }
        sync_frame(base >= cap);
        bound = ub;
        if (K == 0)
            return;
        flags = kFlagSelect;  // a class and v of the smaller frame, in this step
    }

    // Registers (and, for a new frame, class and v) of the frames that need
    // them.  cL then drops v (every child of the frame is split without
    // it), and v's G rows come into registers from HBM, once per frame.
    __device__ void reload() {
        const bool ld = (flags & (kFlagSelect | kFlagLoad)) != 0;
        if (ld)
            load_regs();
        const bool fresh = (flags & kFlagSelect) != 0;
        if (ballot(fresh))
            if (fresh)
                select();
        if (ld) {
            cL &= ~((W)1 << v);
            const W *rows = gadj + (size_t)inst * (NR * NB) + v;
            go = rows[0];
            if constexpr (DIR)
                gi = rows[2 * NB];
        }
        flags &= ~kFlagLoad;
    }

    // Parts of class (L, R) for the child (v, w), by adjacency letter.
    // Part a holds the vertices whose letter is a: bit 0 an edge from v (from
    // w), bit 1 (directed) an edge into v (into w).  A part without a bit is
    // the rest of the part with it (x & ~y == x ^ (x & y)), which saves the
    // complement of each row.
    __device__ void split(W L, W R, W go, W ho, W gi, W hi, W *pl, W *pr) const {
        if constexpr (!DIR) {
            pl[1] = L & go;
            pr[1] = R & ho;
            pl[0] = L ^ pl[1];
            pr[0] = R ^ pr[1];
        } else {
            const W lo1 = L & go, ro1 = R & ho;
            const W lo0 = L ^ lo1, ro0 = R ^ ro1;
            pl[3] = lo1 & gi;
            pr[3] = ro1 & hi;
            pl[1] = lo1 ^ pl[3];
            pr[1] = ro1 ^ pr[3];
            pl[2] = lo0 & gi;
            pr[2] = ro0 & hi;
            pl[0] = lo0 ^ pl[2];
            pr[0] = ro0 ^ pr[2];
        }
    }
    // min(|L_a|, |R_a|) of each part, and their sum.
    DEV int part_mins(const W *pl, const W *pr, int *mn) {
        int s = 0;
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            const int nl = popc(pl[a]), nr = popc(pr[a]);
            mn[a] = nl < nr ? nl : nr;
            s += mn[a];
        }
        return s;
    }

    // The next partner w of v: split, Eq. 1, then prune or descend.
    // (cL no longer holds v: reload() took it out.)
    __device__ void evaluate() {
        const int w = ctz(rrem);
        rrem &= rrem - 1;
        const W wb = (W)1 << w;
        const W ho = sadj[w];
        W hi = 0;
        if constexpr (DIR)
            hi = sadj[arows + w];
        W pl[NR], pr[NR];
        int mn[NR];
        split(cL, cR & ~wb, go, ho, gi, hi, pl, pr);
        int contrib = part_mins(pl, pr, mn);
        if (ballot(K > S) != 0) {  // (rare) classes past the first S
            for (int c = 1; ballot(c * S < K) != 0; ++c) {
                const int k = c * S + lk;
                n_ncls += (unsigned)__builtin_popcount(sbits(ballot(k < K)));
                if (k < K) {
                    const Cls<W> x = cget(base + k);
                    W ql[NR], qr[NR];
                    int qm[NR];
                    split(x.L & ~((W)1 << v), x.R & ~wb, go, ho, gi, hi, ql, qr);
                    contrib += part_mins(ql, qr, qm);
                }
            }
        }
        const int b = d + 1 + ssum(contrib);
        nodes_pend += 1;
        if (b > inc)
            descend(w, b, go, ho, gi, hi, pl, pr, mn);
    }

    // The child (v, w) survived its bound: compact its non-empty classes
    // into a new frame above the top one and make it the top frame.  Every
    // kept class adds at least one to the Eq. 1 sum, so the child has at most
    // b - d - 1 classes: a frame that might not fit below cap starts at cap,
    // in the HBM part of the stack, so no frame straddles the two parts.
    __device__ void descend(int w, int b, W go, W ho, W gi, W hi, const W *pl, const W *pr,
                            const int *mn) {
        int nb = base + K;
        if (nb < cap && nb + (b - d - 1) > cap)
            nb = cap;
        const bool hbm = nb >= cap;
        if (ballot(hbm) != 0) {
            // the HBM part holds hstride classes (none when the LDS part is
            // the whole worst case): a frame past it means a broken invariant
            const bool over = hbm && (long long)(nb - cap + (b - d - 1)) > hstride;
            if (over) {
                if (lk == 0)
                    fail_lane(kErrStack);
                return;
            }
        }
        int K2 = 0;
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            const bool ne = mn[a] != 0;  // both sides non-empty
            const uint32_t m = sbits(ballot(ne));
            const int at = nb + K2 + below(m);
            if (ne) {
                if (!hbm) {
                    scls[2 * at] = pl[a];
                    scls[2 * at + 1] = pr[a];
                } else {
                    hcls[2 * (at - cap)] = pl[a];
                    hcls[2 * (at - cap) + 1] = pr[a];
                }
            }
            K2 += __builtin_popcount(m);
        }
        if (ballot(K > S) != 0) {  // (rare) classes past the first S
            const W vb = (W)1 << v;
            const W wb = (W)1 << w;
            for (int c = 1; ballot(c * S < K) != 0; ++c) {
                const int k = c * S + lk;
                W ql[NR], qr[NR];
                const bool in = k < K;
                const Cls<W> x = cget(base + (in ? k : 0));
                split(in ? x.L & ~vb : (W)0, in ? x.R & ~wb : (W)0, go, ho, gi, hi, ql, qr);
#pragma unroll
                for (int a = 0; a < NR; ++a) {
                    const bool ne = ql[a] != 0 && qr[a] != 0;
                    const uint32_t m = sbits(ballot(ne));
                    const int at = nb + K2 + below(m);
                    if (ne) {
                        if (!hbm) {
                            scls[2 * at] = ql[a];
                            scls[2 * at + 1] = qr[a];
                        } else {
                            hcls[2 * (at - cap)] = ql[a];
                            hcls[2 * (at - cap) + 1] = qr[a];
                        }
                    }
                    K2 += __builtin_popcount(m);
                }
            }
        }
        // the parent frame, with w gone from its partners
        save_hdr(w);
        if (lk == 0)
            smap[d] = (uint16_t)(v | (w << 8));
        sync_frame(hbm);
        if (d + 1 > inc)
            improve(d + 1);
        if (K2 == 0)
            return;  // a leaf: nothing left to split
        if (nb + K2 > max_used)
            max_used = nb + K2;
        if (hbm)
            n_hbm += 1;
        pushed += (unsigned long long)K2;
        t += 1;
        base = nb;
        K = K2;
        d += 1;
        bound = b;
        rrem = 0;
        flags = kFlagSelect;  // class and v at the next step's reload
    }

    // One lock-step search step of every segment that holds a unit.
    // A segment with no unit, or whose unit has finished, has t = -1,
    // rrem = 0 and flags = 0, so the phase tests need not look at inst or fin.
    __device__ void step() {
        const bool need_pop = t >= 0 && rrem == 0 && !(flags & (kFlagUnmatched | kFlagSelect));
        if (ballot(need_pop))
            if (need_pop)
                pop();
        const bool need_unm = rrem == 0 && (flags & kFlagUnmatched);
        if (ballot(need_unm))
            if (need_unm)
                unmatched();
        if (ballot((flags & (kFlagSelect | kFlagLoad)) != 0))
            reload();
        const uint64_t ev = ballot(rrem != 0);
        if (ev) {
            // statistics (wave-uniform): children evaluated, and the lanes
            // holding one of their classes in the first pass
            n_evals += (unsigned)__builtin_popcountll(ev & kLeadLanes);
            n_lanes += (unsigned)__builtin_popcountll(ev & ballot(lk < K));
            if (rrem != 0)
                evaluate();
        }
        n_steps += 1;
        if (ballot(fin))
            finish_units();
    }


    // ---- work sharing ----

    // A free slot in this XCD's ring, else in the next rings.
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
        ok = rl(ok, 0);
        ring = rl(rr, 0);
        ticket = rl_ull(tk, 0);
        return ok != 0;
    }

    __device__ void raise_flag(unsigned bits) {
        if (lane == 0) {
            if (bits & kFlagStop)
                __hip_atomic_store(&P.g->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int k = 0; k < kRings; ++k)
                __hip_atomic_fetch_or(&P.g->xcd[k].flag, bits, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // A check failed in the lanes that call this (any lanes, also inside a
    // divergent branch): record the error and stop every search; the
    // wavefronts leave at their next check().
    __device__ void fail_lane(unsigned code) {
        __hip_atomic_store(&P.g->error, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&P.g->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int k = 0; k < kRings; ++k)
            __hip_atomic_fetch_or(&P.g->xcd[k].flag, kFlagStop, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }

    // Give segment j's shallowest open frame's remaining children to the
    // queue (the frame keeps the rest; the top frame keeps half).
    __device__ void donate(int j) {
        const int jt = of(t, j);
        const uint2 *h = hdr_of(j);
        int b = -1;
        W grr = 0;
        int gfl = 0;
        for (int i = 0; i < jt; ++i) {
            const uint2 x = h[i];
            const uint32_t hx = sc(x.x), hy = sc(x.y);
            if ((int)((hx >> 19) & 0x7Fu) > P.donate_depth)
                return;  // deeper frames hold too little work to hand out
            const uint32_t lo1 = (hy >> 14) & 0x7Fu;
            const int f = (int)((hy >> 13) & 1u);
            W r = 0;
            if (lo1 < (uint32_t)NB) {
                const int fb = (int)(hx & 0xFFFu), fs = (int)(hy & 0x3Fu);
                r = partner_range(sc(cget_of(j, fb + fs).R), lo1, i == 0 ? of(hi0, j) : NB);
            }
            if (r != 0 || (f & kFlagUnmatched)) {
                b = i;
                grr = r;
                gfl = f & kFlagUnmatched;
                break;
            }
        }
        W keep_r = 0;
        const W jr = ofw(rrem, j);
        const int jf = of(flags, j);
        if (b < 0) {
            if (of(d, j) > P.donate_depth)
                return;
            const int n = popc(jr);
            if (n >= 2) {
                // the record takes the lower n/2 partners, the frame keeps
                // the upper ones (so its partners stay R_sel above a vertex)
                W r = jr, low = 0;
                for (int c = 0; c < n / 2; ++c) {
                    low |= r & (~r + 1);
                    r &= r - 1;
                }
                grr = low;
                gfl = jf & kFlagUnmatched;
                keep_r = r;
            } else if (n == 1 && (jf & kFlagUnmatched)) {
                grr = 0;
                gfl = kFlagUnmatched;
                keep_r = jr;
            } else {
                return;
            }
            b = jt;
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
        int fsel;
        if (b == jt) {
            fK = of(K, j);
            fd = of(d, j);
            fbase = of(base, j);
            fsel = of(sel, j);
            rh.v = (uint8_t)of(v, j);
            rh.bound = (uint8_t)of(bound, j);
        } else {
            const uint2 x = h[b];
            const uint32_t hx = sc(x.x), hy = sc(x.y);
            fbase = (int)(hx & 0xFFFu);
            fK = (int)((hx >> 12) & 0x7Fu);
            fd = (int)((hx >> 19) & 0x7Fu);
            rh.v = (uint8_t)(hx >> 26);
            fsel = (int)(hy & 0x3Fu);
            rh.bound = (uint8_t)((hy >> 6) & 0x7Fu);
        }
        rh.sel = (uint8_t)fsel;
        {
            const Cls<W> cs = cget_of(j, fbase + fsel);
            rh.lsel = (uint8_t)popc(sc(cs.L));
            rh.rsel = (uint8_t)popc(sc(cs.R));
        }
        const int ji = of(inst, j);
        rh.inst = (uint32_t)ji;
        rh.K = (uint8_t)fK;
        rh.d = (uint8_t)fd;
        rh.flags = (uint8_t)gfl;
        rh.pad[0] = rh.pad[1] = rh.pad[2] = rh.pad[3] = 0;
        rh.rrem = grr;
        if (lane == 0)
            *(RecHdr<W> *)slot = rh;
        uint16_t *rmap = (uint16_t *)(slot + rec_map_off<W>());
        Cls<W> *rcls = (Cls<W> *)(slot + rec_cls_off<W>());
        const uint16_t *jm = map_of(j);
        for (int i = lane; i < fd; i += 64)
            rmap[i] = jm[i];
        for (int i = lane; i < fK; i += 64)
            rcls[i] = cget_of(j, fbase + i);
        if (lane == 0) {
            a_add_rlx(&P.open[ji], 1);
            a_add_rlx(&P.g->open_total, 1);
            st_rel(&P.seq[idx], ticket + 1);
        }
        if (b == jt) {
            if (seg == j) {
                rrem = keep_r;
                flags = 0;
            }
        } else if (lane == 0) {
            // the frame keeps nothing: no partners, no unmatched child
            uint2 *hw = hdr_of(j);
            uint2 x = hw[b];
            x.y = (x.y & ~((0x7Fu << 14) | (1u << 13))) | (kNoPartners << 14);
            hw[b] = x;
        }
        wave_sync();
        n_don += 1;
    }

    // Segment j starts on instance i: its rows, incumbent, and identity.
    __device__ void set_instance(int j, int i) {
        if (of(adj_inst, j) != i) {
            // H's rows (set 1: out; set 3: in) into the segment's LDS
            const W *src = (const W *)P.adj + (size_t)i * NR * NB;
            W *dst = adj_of(j);
            for (int q = lane; q < (NR / 2) * arows; q += 64)
                dst[q] = src[(2 * (q / arows) + 1) * NB + (q % arows)];
        }
        const DevInst di = P.inst[i];
        const int slot = sc((int)di.inc_slot);
        const int tw = sc((int)di.twin);
        const int don = sc((int)di.dead_on);
        int g = 0;
        if (lane == 0) {
            g = ld_rlx(&P.inc[slot]);
            if (tw >= 0 && ld_rlx(&P.open[tw]) == 0 && !ld_rlx(&P.dead[tw]))
                g = 255;  // the twin's search already finished
            if (don && ld_rlx(&P.dead[i]))
                g = 255;  // given up as a dead end
        }
        g = rl(g, 0);
        if (seg == j) {
            adj_inst = i;
            inst = i;
            inc_slot = slot;
            twin = tw;
            dead_on = don;
            map_off = sc((int)di.map_off);
            target = sc((int)di.target);
            inc = 0;
            set_inc(g);
            nodes_pend = 0;
            fin = false;
        }
    }

    // Take a queued node into segment j: from this XCD's ring, else from
    // one other ring, a different one on each call.
    __device__ bool take_record(int j) {
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
        steal_from = rl(steal_from, 0);
        ok = rl(ok, 0);
        if (!ok)
            return false;
        // pairs with the producer's release store of the slot's sequence number
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        hd = rl_ull(hd, 0);
        const int ring = rl(rr, 0);
        const size_t idx = (size_t)ring * P.ring_slots + (size_t)(hd & mask);
        const uint8_t *slot = P.slots + idx * (size_t)P.slot_bytes;
        const RecHdr<W> rh = *(const RecHdr<W> *)slot;
        const int ri = sc((int)rh.inst);
        const int rK = sc((int)rh.K), rd = sc((int)rh.d), rv = sc((int)rh.v);
        const int rsel_ = sc((int)rh.sel), rb = sc((int)rh.bound), rf = sc((int)rh.flags);
        const W rr_ = sc((W)rh.rrem);
        const uint16_t *rmap = (const uint16_t *)(slot + rec_map_off<W>());
        const Cls<W> *rcls = (const Cls<W> *)(slot + rec_cls_off<W>());
        uint16_t mp = 0;
        Cls<W> cc;
        cc.L = 0;
        cc.R = 0;
        if (lane < rd)
            mp = rmap[lane];
        if (lane < rK)
            cc = rcls[lane];
        // every lane's loads of the slot have returned before it is handed back
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0)
            st_rlx(&P.seq[idx], hd + (unsigned long long)P.ring_slots);
        set_instance(j, ri);
        uint16_t *jm = map_of(j);
        Cls<W> *jc = cls_of(j);
        if (lane < rd)
            jm[lane] = mp;
        if (lane < rK)
            jc[lane] = cc;
        wave_sync();
        if (seg == j) {
            t = 0;
            base = 0;
            K = rK;
            d = rd;
            d0 = rd;
            v = rv;
            sel = rsel_;
            bound = rb;
            rrem = rr_;
            hi0 = rr_ != 0 ? NB - clz(rr_) : 0;  // the record's partners end at its highest
            if (bound <= inc) {
                rrem = 0;
                flags = 0;
            } else if (rf & kFlagFresh) {
                rrem = 0;
                flags = kFlagSelect;
            } else {
                flags = (rf & kFlagUnmatched) | (rrem != 0 ? kFlagLoad : 0);
            }
        }
        n_pops += 1;
        return true;
    }

    // Segment j takes the next unstarted instance (its work unit was counted
    // by the reset).
    __device__ bool claim_instance(int j) {
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
        set_instance(j, i);
        const DevInst di = P.inst[i];
        const int k0 = sc((int)di.K0);
        const Cls<W> *rc = (const Cls<W> *)P.rootcls + sc((int)di.cls_off);
        Cls<W> *jc = cls_of(j);
        for (int q = lane; q < k0; q += 64)
            jc[q] = rc[q];
        wave_sync();
        if (seg == j) {
            t = 0;
            base = 0;
            d = 0;
            d0 = 0;
            K = k0;
            load_regs();
            int contrib = 0;
            for (int c = 0; ballot(c * S < K) != 0; ++c) {
                const int k = c * S + lk;
                if (k < K) {
                    const Cls<W> x = c == 0 ? Cls<W>{cL, cR} : cget(base + k);
                    const int nl = popc(x.L), nr = popc(x.R);
                    contrib += nl < nr ? nl : nr;
                }
            }
            bound = ssum(contrib);
            nodes_pend += 1;  // the root
            rrem = 0;
            flags = (K == 0 || bound <= inc) ? 0 : kFlagSelect;
        }
        return true;
    }

    // Units whose stacks emptied: count their nodes and end them.
    __device__ void finish_units() {
        uint64_t fm = ballot(fin && lk == 0);
        while (fm) {
            const int j = ctz(fm) >> LOGS;
            fm &= fm - 1;
            const int ji = of(inst, j);
            const unsigned np = (unsigned)of((int)nodes_pend, j);
            if (lane == 0) {
                a_add64(&P.nodes[ji], (unsigned long long)np);
                if (P.node_limit > 0) {
                    unsigned long long tot = a_add64(&P.g->node_total, np) + np;
                    if ((long long)tot > P.node_limit)
                        raise_flag(kFlagStop);
                }
                if (!stop) {
                    const int r = a_add_rlx(&P.open[ji], -1);
                    if (r == 1)
                        __hip_atomic_store(&P.t_proof[ji], now_ticks(), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (a_add_rlx(&P.g->open_total, -1) == 1)
                        raise_flag(kFlagDone);
                }
            }
            n_nodes_wave += np;
            if (seg == j) {
                inst = -1;
                fin = false;
                nodes_pend = 0;
            }
        }
    }

    // Nodes counted so far, flushed to the instances (for the node limit).
    __device__ void flush_nodes() {
        uint64_t am = ballot(inst >= 0 && lk == 0);
        unsigned long long tot_add = 0;
        while (am) {
            const int j = ctz(am) >> LOGS;
            am &= am - 1;
            const int ji = of(inst, j);
            const unsigned np = (unsigned)of((int)nodes_pend, j);
            if (lane == 0 && np)
                a_add64(&P.nodes[ji], (unsigned long long)np);
            tot_add += np;
            if (seg == j)
                nodes_pend = 0;
        }
        n_nodes_wave += tot_add;
        if (lane == 0 && tot_add && P.node_limit > 0) {
            unsigned long long tot = a_add64(&P.g->node_total, tot_add) + tot_add;
            if ((long long)tot > P.node_limit)
                raise_flag(kFlagStop);
        }
    }

    // Dead-end forecast (paper Sec. IV.A): an instance whose search has gone
    // more than dead_abs nodes -- and, if dead_rel is set, more than dead_rel
    // times the nodes that led to its last improvement -- without raising
    // its incumbent is given up: every search on it prunes from then on, and
    // the host steps the bound.
    __device__ void forecast_dead_ends() {
        if (inst >= 0 && dead_on && lk == 0) {
            const unsigned long long n = ld_rlx(&P.nodes[inst]);
            const unsigned long long b = ld_rlx(&P.best_nodes[inst]);
            const unsigned long long since = n > b ? n - b : 0ull;
            unsigned long long thr = (unsigned long long)P.dead_abs;
            if (P.dead_rel > 0 && (unsigned long long)P.dead_rel * b > thr)
                thr = (unsigned long long)P.dead_rel * b;
            if (since > thr) {
                st_rlx(&P.dead[inst], 1);
                inc = 255;
            }
        }
        inc = sfirst(inc);
    }

    // Periodic: refresh incumbents, honour limits, keep the queue stocked.
    __device__ void check() {
        since_check = 0;
        unsigned fl = 0;
        unsigned long long hd = 0, tl = 0;
        const bool may_donate = !P.single_wave && P.donate_low >= 0;
        if (lane == 0) {
            fl = ld_rlx(&P.g->xcd[my_ring].flag);
            if (may_donate) {
                tl = ld_rlx(&P.g->ring[my_ring].tail);
                hd = ld_rlx(&P.g->ring[my_ring].head);
            }
        }
        if (inst >= 0) {
            int g = ld_rlx(&P.inc[inc_slot]);
            if (twin >= 0 && ld_rlx(&P.open[twin]) == 0 && !ld_rlx(&P.dead[twin]))
                g = 255;
            if (dead_on && ld_rlx(&P.dead[inst]))
                g = 255;
            set_inc(g);
        }
        if (rl(fl, 0)) {
            stop = true;
            return;
        }
        if (now_ticks() - t_start > P.limit_ticks) {
            raise_flag(kFlagStop);
            stop = true;
            return;
        }
        // (counts are also flushed before a 32-bit per-unit count could wrap)
        if (P.node_limit > 0 || P.dead_abs > 0 || ballot(nodes_pend > (1u << 30)))
            flush_nodes();
        if (P.dead_abs > 0)
            forecast_dead_ends();
        if (may_donate) {
            const long long waiting = (long long)(rl_ull(tl, 0) - rl_ull(hd, 0));
            if (waiting < P.donate_low) {
                // one donation per check, from the segments in turn
                const uint64_t cand = ballot(inst >= 0 && !fin && lk == 0 && d0 <= P.donate_depth);
                if (cand) {
                    const uint64_t rot = cand >> (donor << LOGS);
                    const int j = rot ? (ctz(rot) >> LOGS) + donor : ctz(cand) >> LOGS;
                    donor = (j + 1) & (NSEG - 1);
                    donate(j);
                }
            }
        }
    }

    // Give idle segments work; false if none was found.
    __device__ bool refill() {
        uint64_t im = ballot(inst < 0 && lk == 0);
        if (P.single_wave)
            im &= 1ull;  // one search only: the sequential order
        bool any = false;
        while (im) {
            const int j = ctz(im) >> LOGS;
            im &= im - 1;
            bool got = false;
            if (!P.single_wave)
                got = take_record(j);
            if (!got)
                got = claim_instance(j);
            if (!got)
                break;
            any = true;
        }
        return any;
    }

    __device__ void main_loop() {
        t_start = now_ticks();
        if (lane == 0)
            a_min64(&P.g->t0, t_start);
        int backoff = 0;
        int idle_steps = 0;
        int refill_gap = 16;  // steps between refills while some segments are busy
        unsigned long long t_busy0 = 0;
        bool busy = false;
        for (;;) {
            // idle segments look for work when the wavefront has none at all,
            // and otherwise every few steps
            // (a failed look costs the busy segments a queue round trip, so
            // the gap doubles while the queue stays empty)
            const uint64_t am = ballot(inst >= 0);
            if (am == 0 || (am != ~0ull && ++idle_steps >= refill_gap)) {
                idle_steps = 0;
                if (refill())
                    refill_gap = 16;
                else if (am != 0)
                    refill_gap = refill_gap < 1024 ? 2 * refill_gap : 1024;
            }
            if (ballot(inst >= 0) == 0) {
                if (busy) {
                    n_busy += now_ticks() - t_busy0;
                    busy = false;
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
                const int bmax = P.backoff_max;
                backoff = backoff ? (2 * backoff < bmax ? 2 * backoff : bmax) : 1;
                const unsigned long long t_sleep = now_ticks();
                for (int i = 0; i < backoff; ++i)
                    __builtin_amdgcn_s_sleep(127);
                n_sleep += now_ticks() - t_sleep;
                continue;
            }
            backoff = 0;
            if (!busy) {
                t_busy0 = now_ticks();
                busy = true;
            }
            step();
            if (stop)
                break;
            if (++since_check >= check_interval) {
                check();
                if (stop)
                    break;
            }
        }
        if (busy)
            n_busy += now_ticks() - t_busy0;
        // classes pushed and frames placed in HBM, summed over the segments
        // (lane 0 of each)
        n_pushed = seg_total(pushed);
        n_hbm = seg_total(n_hbm);
        n_ncls = seg_total(n_ncls);
        if (lane == 0) {
            a_add64(&P.g->batches, n_steps);
            a_add64(&P.g->children, n_evals);
            a_add64(&P.g->lane_slots, n_lanes);
            a_add64(&P.g->donations, n_don);
            a_add64(&P.g->pops, n_pops);
            a_add64(&P.g->busy_ticks, n_busy);
            a_add64(&P.g->hbm_frames, n_hbm);
            a_add64(&P.g->pushed_classes, n_pushed);
            a_add64(&P.g->sleep_ticks, n_sleep);
            a_add64(&P.g->node_classes, n_lanes + n_ncls);
        }
        const int mu = wave_max_i(max_used);
        if (lane == 0)
            __hip_atomic_fetch_max(&P.g->max_stack, mu, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }

    DEV int wave_max_i(int x) { return (int)~wave_min(~(uint32_t)x); }
    __device__ unsigned long long seg_total(unsigned long long x) const {
        x = lk == 0 ? x : 0ull;
        return (unsigned long long)(unsigned)wave_sum((int)(unsigned)x) +
               ((unsigned long long)(unsigned)wave_sum((int)(unsigned)(x >> 32)) << 32);
    }
};

template <typename W, bool DIR, int LOGS>
__global__ void __launch_bounds__(256) mcs_seg_kernel(SearchParams Pk) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ SearchParams P;
    if (threadIdx.x == 0)
        P = Pk;
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    if (Pk.single_wave && (blockIdx.x != 0 || wv != 0))
        return;
    SegSearch<W, DIR, LOGS> s(P, smem + (size_t)wv * (size_t)(Pk.seg_bytes * (64 >> LOGS)),
                              (long long)blockIdx.x * (blockDim.x >> 6) + wv);
    s.main_loop();
}

}  // namespace mcs

// Launch entry point used by the host driver: the kernel for rows of
// word_bytes (4 or 8), directed or not, with segments of 2^seg_log lanes
// (2, 3 or 4); null for anything else.
extern "C" void *mcs_internal_seg_kernel(int word_bytes, int directed, int seg_log) {
    using namespace mcs;
    if (seg_log == 2)
        return word_bytes == 4 ? (directed ? (void *)mcs_seg_kernel<uint32_t, true, 2>
                                           : (void *)mcs_seg_kernel<uint32_t, false, 2>)
               : word_bytes == 8 ? (directed ? (void *)mcs_seg_kernel<uint64_t, true, 2>
                                             : (void *)mcs_seg_kernel<uint64_t, false, 2>)
                                 : nullptr;
    if (word_bytes == 4) {
        if (seg_log == 3)
            return directed ? (void *)mcs_seg_kernel<uint32_t, true, 3>
                            : (void *)mcs_seg_kernel<uint32_t, false, 3>;
        if (seg_log == 4)
            return directed ? (void *)mcs_seg_kernel<uint32_t, true, 4>
                            : (void *)mcs_seg_kernel<uint32_t, false, 4>;
    } else if (word_bytes == 8) {
        if (seg_log == 3)
            return directed ? (void *)mcs_seg_kernel<uint64_t, true, 3>
                            : (void *)mcs_seg_kernel<uint64_t, false, 3>;
        if (seg_log == 4)
            return directed ? (void *)mcs_seg_kernel<uint64_t, true, 4>
                            : (void *)mcs_seg_kernel<uint64_t, false, 4>;
    }
    return nullptr;
}
