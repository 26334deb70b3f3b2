// The 3D Hilbert curve of the key stage as a finite state machine (shared by
// the key kernels, which encode, and the focused-tree MAC, which decodes node
// keys into grid boxes).
#pragma once

#include <cstdint>

namespace cs {

// ---- Hilbert curve as a state machine -----------------------------------
//
// Skilling's transform (AIP Conf. Proc. 707, 2004) visits the bit planes from
// the top. At each plane it either reflects the lower bits of word 0 or swaps
// the lower bits of word 0 and word i, so everything it does to the lower planes
// is an axis permutation plus reflection (a symmetry of the cube). Its Gray
// stage is local to a plane, up to a running parity that complements every
// later digit. The key digit of a plane is therefore a function of the plane's
// raw octant and a state (axis permutation, reflection mask, parity); the
// state reachable from the identity are enumerated here at compile time.

struct HState {
    uint8_t perm[3];  // transformed axis a reads raw axis perm[a]
    uint8_t mask;     // reflection of transformed axis a in bit a
    uint8_t parity;
};

constexpr bool same(const HState& a, const HState& b) {
    return a.perm[0] == b.perm[0] && a.perm[1] == b.perm[1] && a.perm[2] == b.perm[2] && a.mask == b.mask &&
           a.parity == b.parity;
}

// One bit plane: raw octant o = 4x + 2y + z -> key digit, next state.
constexpr uint32_t plane_step(const HState& s, uint32_t o, HState& next) {
    uint32_t raw[3] = {(o >> 2) & 1u, (o >> 1) & 1u, o & 1u};
    uint32_t w[3] = {};
    for (int a = 0; a < 3; ++a) w[a] = raw[s.perm[a]] ^ ((s.mask >> a) & 1u);
    uint32_t g0 = w[0], g1 = w[1] ^ w[0], g2 = w[2] ^ w[1] ^ w[0];
    uint32_t digit = (g0 << 2) | (g1 << 1) | g2;
    if (s.parity) digit ^= 7u;
    uint8_t p[3] = {s.perm[0], s.perm[1], s.perm[2]};
    uint8_t m[3] = {static_cast<uint8_t>(s.mask & 1u), static_cast<uint8_t>((s.mask >> 1) & 1u),
                    static_cast<uint8_t>((s.mask >> 2) & 1u)};
    for (int i = 0; i < 3; ++i) {
        if (w[i]) {
            m[0] ^= 1u;
        } else {
            uint8_t tp = p[0];
            p[0] = p[i];
            p[i] = tp;
            uint8_t tm = m[0];
            m[0] = m[i];
            m[i] = tm;
        }
    }
    next = HState{{p[0], p[1], p[2]}, static_cast<uint8_t>(m[0] | (m[1] << 1) | (m[2] << 2)),
                  static_cast<uint8_t>(s.parity ^ g2)};
    return digit;
}

constexpr int kMaxStates = 96;
constexpr int kStates = 48;  // reachable states (checked below)

struct HilbertTables {
    // one plane from the start state: digit | next << 3
    uint16_t first[8];
    // two planes: index = state * 64 + (octant_hi << 3 | octant_lo),
    // entry = (digit_hi << 3 | digit_lo) | next << 6
    uint16_t two[kStates * 64];
    int count;
};

constexpr HilbertTables make_tables() {
    HState st[kMaxStates] = {};
    uint16_t one[kMaxStates][8] = {};
    int count = 1;
    st[0] = HState{{0, 1, 2}, 0, 0};
    for (int s = 0; s < count; ++s) {
        for (uint32_t o = 0; o < 8; ++o) {
            HState nx{};
            uint32_t d = plane_step(st[s], o, nx);
            int idx = -1;
            for (int k = 0; k < count; ++k)
                if (same(st[k], nx)) idx = k;
            if (idx < 0) {
                idx = count;
                st[count++] = nx;
            }
            one[s][o] = static_cast<uint16_t>(d | (idx << 3));
        }
    }
    HilbertTables t{};
    t.count = count;
    for (int o = 0; o < 8; ++o) t.first[o] = one[0][o];
    for (int s = 0; s < kStates && s < count; ++s)
        for (uint32_t o = 0; o < 64; ++o) {
            uint32_t e1 = one[s][o >> 3];
            uint32_t e2 = one[e1 >> 3][o & 7u];
            t.two[s * 64 + o] = static_cast<uint16_t>(((e1 & 7u) << 3) | (e2 & 7u) | ((e2 >> 3) << 6));
        }
    return t;
}

constexpr HilbertTables kHilbert = make_tables();
static_assert(kHilbert.count == kStates, "unexpected number of Hilbert states");

// Decoding: for state s and key digit d, the raw octant (4x + 2y + z) and the
// next state, entry = octant | next << 3 (the inverse of the one-plane table).
struct HilbertDecode {
    uint16_t dec[kStates * 8];
};

constexpr HilbertDecode make_decode() {
    HState st[kMaxStates] = {};
    uint16_t one[kMaxStates][8] = {};
    int count = 1;
    st[0] = HState{{0, 1, 2}, 0, 0};
    for (int s = 0; s < count; ++s) {
        for (uint32_t o = 0; o < 8; ++o) {
            HState nx{};
            uint32_t d = plane_step(st[s], o, nx);
            int idx = -1;
            for (int k = 0; k < count; ++k)
                if (same(st[k], nx)) idx = k;
            if (idx < 0) {
                idx = count;
                st[count++] = nx;
            }
            one[s][o] = static_cast<uint16_t>(d | (idx << 3));
        }
    }
    HilbertDecode t{};
    for (int s = 0; s < kStates && s < count; ++s)
        for (uint32_t o = 0; o < 8; ++o) t.dec[s * 8 + (one[s][o] & 7u)] = static_cast<uint16_t>(o | ((one[s][o] >> 3) << 3));
    return t;
}

constexpr HilbertDecode kHilbertDecode = make_decode();

// Lower corner of the grid box of the node whose keys start at `start` on
// `level` (its first `level` octal digits fix the box; edge 2^(L - level)).
// curve: CSTONE_MORTON (digits are raw octants) or CSTONE_HILBERT.
__host__ __device__ inline void node_corner(uint64_t start, int level, int curve, const uint16_t* dec,
                                            uint32_t corner[3]) {
    uint32_t x = 0, y = 0, z = 0, state = 0;
    for (int l = 1; l <= level; ++l) {
        const uint32_t d = static_cast<uint32_t>(start >> (63 - 3 * l)) & 7u;
        uint32_t o = d;
        if (curve == 1) {
            const uint32_t e = dec[state * 8 + d];
            o = e & 7u;
            state = e >> 3;
        }
        x = (x << 1) | ((o >> 2) & 1u);
        y = (y << 1) | ((o >> 1) & 1u);
        z = (z << 1) | (o & 1u);
    }
    const int sh = 21 - level;
    corner[0] = level ? x << sh : 0u;
    corner[1] = level ? y << sh : 0u;
    corner[2] = level ? z << sh : 0u;
}

}  // namespace cs
