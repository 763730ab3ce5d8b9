// Device helpers shared by the search kernels (mcs_search.hip, one search
// per wavefront, and mcs_seg.hip, one search per lane segment): bit and
// wave helpers, agent-scope atomics, and the queued node record.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <hip/hip_fp16.h>

#include "mcs_layout.h"

namespace mcs {

#define DEV static __device__ __forceinline__

// Rows of graphs with 65..128 vertices.
using u128 = unsigned __int128;

// Rows of graphs with 129..254 vertices: four 64-bit words, low word first.
// The integer operators the search applies to a row word (bitwise logic,
// shifts, and the x - 1 / ~x + 1 of lowest-bit tricks) are written out per
// word; a shift count is at most 255.
struct u256 {
    uint64_t w[4];
    u256() = default;
    __host__ __device__ constexpr u256(uint64_t x) : w{x, 0, 0, 0} {}
    __device__ explicit operator bool() const { return (w[0] | w[1] | w[2] | w[3]) != 0; }
    __device__ explicit operator uint64_t() const { return w[0]; }
    __device__ explicit operator uint32_t() const { return (uint32_t)w[0]; }
    __device__ explicit operator int() const { return (int)w[0]; }
};
__device__ __forceinline__ u256 operator&(const u256 &a, const u256 &b) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = a.w[i] & b.w[i];
    return r;
}
__device__ __forceinline__ u256 operator|(const u256 &a, const u256 &b) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = a.w[i] | b.w[i];
    return r;
}
__device__ __forceinline__ u256 operator^(const u256 &a, const u256 &b) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = a.w[i] ^ b.w[i];
    return r;
}
__device__ __forceinline__ u256 operator~(const u256 &a) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = ~a.w[i];
    return r;
}
__device__ __forceinline__ u256 &operator&=(u256 &a, const u256 &b) { return a = a & b; }
__device__ __forceinline__ u256 &operator|=(u256 &a, const u256 &b) { return a = a | b; }
__device__ __forceinline__ u256 &operator^=(u256 &a, const u256 &b) { return a = a ^ b; }
__device__ __forceinline__ bool operator==(const u256 &a, const u256 &b) {
    return ((a.w[0] ^ b.w[0]) | (a.w[1] ^ b.w[1]) | (a.w[2] ^ b.w[2]) | (a.w[3] ^ b.w[3])) == 0;
}
__device__ __forceinline__ bool operator!=(const u256 &a, const u256 &b) { return !(a == b); }
__device__ __forceinline__ u256 operator+(const u256 &a, const u256 &b) {
    u256 r;
    uint64_t c = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t s = a.w[i] + b.w[i];
        const uint64_t t = s + c;
        c = (uint64_t)(s < a.w[i]) | (uint64_t)(t < s);
        r.w[i] = t;
    }
    return r;
}
__device__ __forceinline__ u256 operator-(const u256 &a, const u256 &b) { return a + (~b + u256(1)); }
// Word j of the result takes words j - q and j - q - 1 of a (q = s / 64).
__device__ __forceinline__ u256 operator<<(const u256 &a, int s) {
    const int q = s >> 6, b = s & 63;
    u256 r;
    for (int j = 0; j < 4; ++j) {
        uint64_t hi = 0, lo = 0;
        for (int i = 0; i < 4; ++i) {
            hi = (j - i == q) ? a.w[i] : hi;
            lo = (j - i == q + 1) ? a.w[i] : lo;
        }
        r.w[j] = (hi << b) | (b ? lo >> (64 - b) : 0);
    }
    return r;
}
__device__ __forceinline__ u256 operator>>(const u256 &a, int s) {
    const int q = s >> 6, b = s & 63;
    u256 r;
    for (int j = 0; j < 4; ++j) {
        uint64_t lo = 0, hi = 0;
        for (int i = 0; i < 4; ++i) {
            lo = (i - j == q) ? a.w[i] : lo;
            hi = (i - j == q + 1) ? a.w[i] : hi;
        }
        r.w[j] = (lo >> b) | (b ? hi << (64 - b) : 0);
    }
    return r;
}

template <typename W>
struct Cls {
    W L, R;
};

// A row word or class in memory (LDS, HBM stack or queued record), read
// and written word by word: an aggregate copy of a 256-bit value goes
// through a temporary in scratch memory.
template <typename W>
DEV W ld_w(const W *p) {
    if constexpr (sizeof(W) == 32) {
        const uint64_t *q = (const uint64_t *)p;
        W x;
        for (int i = 0; i < 4; ++i)
            x.w[i] = q[i];
        return x;
    } else {
        return *p;
    }
}
template <typename W>
DEV void st_w(W *p, const W &x) {
    if constexpr (sizeof(W) == 32) {
        uint64_t *q = (uint64_t *)p;
        for (int i = 0; i < 4; ++i)
            q[i] = x.w[i];
    } else {
        *p = x;
    }
}
template <typename W>
DEV Cls<W> ld_cls(const Cls<W> *p) {
    Cls<W> c;
    c.L = ld_w(&p->L);
    c.R = ld_w(&p->R);
    return c;
}
template <typename W>
DEV void st_cls(Cls<W> *p, const Cls<W> &c) {
    st_w(&p->L, c.L);
    st_w(&p->R, c.R);
}

// A frame header in LDS: one 32-bit word per field, written from lane f of
// one register (v_writelane, then a single masked LDS store) and read back
// with one LDS load and v_readlane -- no byte packing on the scalar unit.
enum HdrField {
    kHRremLo = 0,  // children (w of the selected class) not yet taken
    kHRremHi,
    kHBase,        // first class of the frame in the LDS class stack
    kHK,
    kHD,
    kHV,
    kHSel,
    kHBound,
    kHFlags,
    kHLsel,
    kHRsel,
    kHRrem2,  // (128-bit rows) bits 64..95 and 96..127 of the partner mask
    kHRrem3,
    kHRrem4,  // (256-bit rows) bits 128..255 of the partner mask
    kHRrem5,
    kHRrem6,
    kHRrem7,
};

// Header field of bits 32k..32k+31 of the partner mask.
constexpr int rrem_field(int k) { return k < 2 ? k : kHRrem2 + (k - 2); }

template <typename W>
struct RecHdr {
    uint32_t inst;
    uint8_t K, d, v, sel, bound, flags, lsel, rsel;
    uint8_t pad[4];
    W rrem;
};

static_assert(kHRsel < kHdrWords && kHRrem3 < kHdrWordsWide && kHRrem7 < kHdrWords256,
              "header layout");
static_assert(sizeof(RecHdr<uint64_t>) <= rec_header(8) && sizeof(RecHdr<uint32_t>) <= rec_header(4) &&
                  sizeof(RecHdr<u128>) <= rec_header(16) && sizeof(RecHdr<u256>) <= rec_header(32),
              "record header layout");

constexpr int kFlagUnmatched = 1;  // the "v unmatched" child is still to do
constexpr int kFlagOrdered = 2;    // partners are tried in the policy's order
constexpr int kFlagFresh = 4;      // (records only) a child whose class and v are not chosen yet

// ---- bit helpers -----------------------------------------------------------

DEV int popc(uint32_t x) { return __builtin_popcount(x); }
DEV int popc(uint64_t x) { return __builtin_popcountll(x); }
DEV int ctz(uint32_t x) { return __builtin_ctz(x); }
DEV int ctz(uint64_t x) { return __builtin_ctzll(x); }
DEV int clz(uint32_t x) { return __builtin_clz(x); }
DEV int clz(uint64_t x) { return __builtin_clzll(x); }

DEV int popc(u128 x) { return popc((uint64_t)x) + popc((uint64_t)(x >> 64)); }
DEV int ctz(u128 x) {
    const uint64_t lo = (uint64_t)x;
    return lo ? ctz(lo) : 64 + ctz((uint64_t)(x >> 64));
}
DEV int popc(const u256 &x) { return popc(x.w[0]) + popc(x.w[1]) + popc(x.w[2]) + popc(x.w[3]); }
DEV int ctz(const u256 &x) {
    return x.w[0] ? ctz(x.w[0])
           : x.w[1] ? 64 + ctz(x.w[1])
           : x.w[2] ? 128 + ctz(x.w[2])
                    : 192 + ctz(x.w[3]);
}

// 64-bit word q of a row word (zero past its width), and a row word from
// its 64-bit words.
DEV uint64_t word64(uint32_t x, int q) { return q == 0 ? x : 0; }
DEV uint64_t word64(uint64_t x, int q) { return q == 0 ? x : 0; }
DEV uint64_t word64(u128 x, int q) { return q == 0 ? (uint64_t)x : q == 1 ? (uint64_t)(x >> 64) : 0; }
DEV uint64_t word64(const u256 &x, int q) { return q < 4 ? x.w[q] : 0; }
template <typename W>
DEV W from_words(const uint64_t *x) {
    if constexpr (sizeof(W) == 32) {
        u256 r;
        for (int i = 0; i < 4; ++i)
            r.w[i] = x[i];
        return r;
    } else if constexpr (sizeof(W) == 16) {
        return ((u128)x[1] << 64) | x[0];
    } else {
        return (W)x[0];
    }
}
// c ? a : b on row words.  For u256 the choice is made per word: a
// conditional on two struct lvalues selects between their addresses, which
// would keep the registers of a search's row words in scratch memory.
template <typename W>
DEV W pick(bool c, const W &a, const W &b) {
    if constexpr (sizeof(W) == 32) {
        u256 r;
        for (int i = 0; i < 4; ++i)
            r.w[i] = c ? a.w[i] : b.w[i];
        return r;
    } else {
        return c ? a : b;
    }
}
// Bit i of a row word, as a row word.
template <typename W>
DEV W bit_at(int i) {
    if constexpr (sizeof(W) == 32) {
        u256 r;
        for (int j = 0; j < 4; ++j)
            r.w[j] = (i >> 6) == j ? 1ull << (i & 63) : 0;
        return r;
    } else {
        return (W)1 << i;
    }
}
template <typename W>
DEV bool test_bit(const W &x, int i) {
    if constexpr (sizeof(W) == 32) {
        const uint64_t a = (i >> 6) == 0 ? x.w[0] : (i >> 6) == 1 ? x.w[1] : (i >> 6) == 2 ? x.w[2] : x.w[3];
        return (a >> (i & 63)) & 1;
    } else {
        return (x >> i) & 1;
    }
}

// ---- wave helpers ----------------------------------------------------------

DEV int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

DEV int sc(int x) { return __builtin_amdgcn_readfirstlane(x); }
DEV uint32_t sc(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
DEV uint64_t sc(uint64_t x) {
    uint32_t lo = sc((uint32_t)x), hi = sc((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
DEV int rl(int x, int l) { return __builtin_amdgcn_readlane(x, l); }
DEV uint32_t rl(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }
DEV uint64_t rl(uint64_t x, int l) {
    uint32_t lo = rl((uint32_t)x, l), hi = rl((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
DEV unsigned long long rl_ull(unsigned long long x, int l) { return (unsigned long long)rl((uint64_t)x, l); }
DEV u128 sc(u128 x) { return ((u128)sc((uint64_t)(x >> 64)) << 64) | sc((uint64_t)x); }
DEV u128 rl(u128 x, int l) { return ((u128)rl((uint64_t)(x >> 64), l) << 64) | rl((uint64_t)x, l); }
DEV u256 sc(const u256 &x) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = sc(x.w[i]);
    return r;
}
DEV u256 rl(const u256 &x, int l) {
    u256 r;
    for (int i = 0; i < 4; ++i)
        r.w[i] = rl(x.w[i], l);
    return r;
}

DEV uint64_t ballot(bool p) { return __ballot(p); }
DEV int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

template <int CTRL>
DEV int dpp(int x) { return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false); }

// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140: all lanes of an 8-lane
// (resp. 16-lane) group end with the group's sum.
DEV int sum8(int x) {
    x += dpp<0xB1>(x);
    x += dpp<0x4E>(x);
    x += dpp<0x141>(x);
    return x;
}
DEV int sum16(int x) {
    x = sum8(x);
    x += dpp<0x140>(x);
    return x;
}
DEV int wave_sum(int x) {
    int s = sum16(x);
    return rl(s, 0) + rl(s, 16) + rl(s, 32) + rl(s, 48);
}
DEV uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Segmented reductions over segments of 2^logS lanes.  The result is valid
// in the last lane of each segment (lane (c << logS) + 2^logS - 1); for
// logS <= 4 every lane of a segment holds it.  row_bcast:15 (0x142) adds
// lane 15 of each row into the next row (rows 1 and 3 enabled), and
// row_bcast:31 (0x143) adds lane 31 into rows 2 and 3.
DEV int seg_sum(int x, int logS) {
    x = sum8(x);
    if (logS >= 4)
        x += dpp<0x140>(x);
    if (logS >= 5)
        x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);
    if (logS >= 6)
        x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);
    return x;
}
template <int CTRL, int ROWS>
DEV uint32_t dpp_min_id(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, CTRL, ROWS, 0xF, false);
}
// Minimum over the first segment (lanes 0 .. 2^logS - 1), as a scalar.
DEV uint32_t seg0_min(uint32_t x, int logS) {
    x = umin(x, (uint32_t)dpp<0xB1>((int)x));
    x = umin(x, (uint32_t)dpp<0x4E>((int)x));
    x = umin(x, (uint32_t)dpp<0x141>((int)x));
    if (logS >= 4)
        x = umin(x, (uint32_t)dpp<0x140>((int)x));
    if (logS >= 5)
        x = umin(x, dpp_min_id<0x142, 0xA>(x));
    if (logS >= 6)
        x = umin(x, dpp_min_id<0x143, 0xC>(x));
    return rl(x, (1 << logS) - 1);
}
DEV uint32_t wave_min(uint32_t x) {
    x = umin(x, (uint32_t)dpp<0xB1>((int)x));
    x = umin(x, (uint32_t)dpp<0x4E>((int)x));
    x = umin(x, (uint32_t)dpp<0x141>((int)x));
    x = umin(x, (uint32_t)dpp<0x140>((int)x));
    return umin(umin(rl(x, 0), rl(x, 16)), umin(rl(x, 32), rl(x, 48)));
}

// Orders LDS traffic between lanes of one wave (LDS executes a wave's
// operations in order; this keeps the compiler from moving them).
DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The same for a wave's stores to global memory read back by other lanes of
// the wave: the stores complete (reach the CU's L1 and L2) before any later
// load issues.
DEV void wave_sync_global() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---- device-scope atomics ----------------------------------------------------

// Counters are relaxed: the only data handed between wavefronts is a queued
// node record, ordered by the release/acquire pair on its slot's sequence.
DEV int a_add_rlx(int *p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV unsigned a_addu(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV unsigned long long a_add64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV int a_max(int *p, int v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void a_max64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void a_min64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
DEV T ld_rlx(T *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
DEV void st_rel(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
DEV void st_rlx(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// Ticket claims are relaxed: the data a ticket guards is ordered by the
// slot's sequence number alone (see take_record and reserve).  At agent
// scope an acquire or release costs a write-back or invalidation of the
// XCD's whole L2, so the queue uses exactly one of each per record.
DEV bool cas64(unsigned long long *p, unsigned long long expect, unsigned long long want) {
    return __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DEV unsigned long long now_ticks() { return wall_clock64(); }

DEV float hf(uint16_t h) { return __half2float(__ushort_as_half(h)); }
DEV float rlf(float x, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); }
template <int CTRL>
DEV float fdpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
DEV float fwave_sum(float x) {
    x += fdpp<0xB1>(x);
    x += fdpp<0x4E>(x);
    x += fdpp<0x141>(x);
    x += fdpp<0x140>(x);
    return (rlf(x, 0) + rlf(x, 16)) + (rlf(x, 32) + rlf(x, 48));
}

}  // namespace mcs
