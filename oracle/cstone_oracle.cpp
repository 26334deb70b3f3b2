// Cornerstone octree build: plain single-threaded CPU ORACLE.
//
// TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or load
// this file or the library built from it; only the test suite, the smoke check
// and the benchmark's CPU-baseline leg use it. It shares no code, header, table
// or constant generator with the HIP implementation.
//
// Every function follows the paper (Keller et al., "Cornerstone: Octree
// Construction Algorithms for Scalable Particle Simulations", PASC '23) as
// directly as possible, in the paper's notation, with no blocking, fusion or
// reordering beyond what the definitions state. Where the paper is silent or
// garbled, the reading taken is stated beside the code (R1..R16 in the design
// notes use the same numbering).
//
// Pins (what checks this oracle against something other than itself) live in
// tests/test_oracle_*.py.  Parity status per function:
//   quantize            pinned (closed form on the unit box, box edge cases)
//   morton key          pinned (octant digits, Z-order comparison, bijection)
//   hilbert key         pinned against curve invariants (bijection, unit steps,
//                       aligned octant blocks, origin); parity with the paper's
//                       own Hilbert variant is UNPINNED (the paper does not fix
//                       which 3D Hilbert curve it uses)
//   sort                pinned (full characterisation of a stable sort)
//   node counts         pinned (brute-force linear count)
//   leaves (top-down)   pinned (balance invariants, which fix the tree uniquely;
//                       paper Fig. 1 worked example)
//   one rebalance step  pinned (paper Fig. 1 split, its reverse merge, and
//                       iteration to the top-down fixed point)
//   link                pinned (paper Fig. 2 level offsets, structural
//                       characterisation of NK / CO / LO)
//   octree node counts  pinned (root = N, children sum to their parent,
//                       leaves equal Eq. histogram, brute-force count)
//   SFC partition       pinned (brute-force search of the defining minimum,
//                       balance within one leaf's count, equal-count cases)
//   focus MAC           pinned (brute force over F's cells at a coarse
//                       level, translation and reflection cases, overlap)
//   focused leaves      pinned (theta = 0 and F = whole domain reduce to the
//                       balanced tree; Sec. 7.1 definition checked leaf by
//                       leaf; the literal g^LE iteration reaches it)
//   compact octree      pinned (without empty leaves it is the linked
//                       octree; every internal node has 2 or more children;
//                       parents contain their children; brute force on
//                       tiny trees)
//   radix nodes         pinned (brute force over all key pairs; ranges nest
//                       and every key has one parent; the nodes with prefix
//                       length 3 l are exactly the internal octree nodes)
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC (no fast-math).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

namespace {

constexpr int kL = 21;                         // octal digits per key (Sec. 3: L = 21 for 64-bit words)
constexpr uint64_t kRootEnd = 1ull << 63;      // 8^L, the last entry of every cornerstone array (Eq. cstone)
constexpr uint32_t kGridMax = (1u << kL) - 1;  // largest integer grid coordinate

// 8^e for 0 <= e <= 21.
uint64_t pow8(int e) { return 1ull << (3 * e); }

// Division level of a node covering a key range of length delta = 8^(L-level)
// (Sec. 4: the i-th leaf has level L - log8(delta_i)).
int level_of_span(uint64_t delta) {
    int e = 0;
    while (pow8(e) < delta) ++e;
    return kL - e;
}

// ---- Coordinates -> integer grid (reading R1; the paper is silent) ---------
//
// t = (c - lo) * s with s = 2^L / (hi - lo), each operation one IEEE double
// rounding; t is clamped to [0, 2^L - 1] and truncated (floor for t >= 0). A
// NaN lands on 0 (it fails t >= 0), +Inf on 2^L - 1. The caller learns about
// non-finite coordinates from the return flag.
uint32_t quantize_one(double c, double lo, double s) {
    double t = (c - lo) * s;
    if (!(t >= 0.0)) return 0;
    if (t >= 2097152.0) return kGridMax;  // 2^21
    return static_cast<uint32_t>(t);
}

// ---- Morton Z-curve key (Sec. 3; reading R2: x is the most significant bit of
// every octal digit). Written straight from the definition
//   key = sum_b 8^b * (4 x_b + 2 y_b + z_b).
uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz) {
    uint64_t key = 0;
    for (int b = 0; b < kL; ++b) {
        uint64_t digit = 4u * ((ix >> b) & 1u) + 2u * ((iy >> b) & 1u) + ((iz >> b) & 1u);
        key += digit << (3 * b);
    }
    return key;
}

// ---- 3D Hilbert key (reading R3): J. Skilling, "Programming the Hilbert
// curve", AIP Conf. Proc. 707 (2004). Coordinates are turned into the
// "transposed" Hilbert index by the two published stages (undo the excess work
// from the top bit plane down, then Gray-encode), and the transposed words are
// interleaved with word 0 (x) as the most significant bit of each octal digit.
uint64_t hilbert(uint32_t ix, uint32_t iy, uint32_t iz, int bits) {
    uint32_t X[3] = {ix, iy, iz};
    const uint32_t top = 1u << (bits - 1);
    // Stage 1: for every bit plane Q from the top down to the second lowest,
    // either reflect the lower bits of X[0] or exchange them with X[i].
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        const uint32_t low = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= low;
            } else {
                uint32_t t = (X[0] ^ X[i]) & low;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    // Stage 2: Gray encode across the three words ...
    X[1] ^= X[0];
    X[2] ^= X[1];
    // ... and fold the running parity of the last word into every word.
    uint32_t flip = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[2] & Q) flip ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= flip;
    // Interleave: bit plane by bit plane from the top, X[0] first.
    uint64_t key = 0;
    for (int q = bits - 1; q >= 0; --q)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> q) & 1u);
    return key;
}

// Inverse of hilbert(): the published decoder (Gray decode, then redo the
// exchanges/reflections from the second lowest bit plane up). Used only by
// tests to check the curve's invariants.
void hilbert_decode(uint64_t key, int bits, uint32_t out[3]) {
    uint32_t X[3] = {0, 0, 0};
    for (int q = bits - 1; q >= 0; --q)
        for (int i = 0; i < 3; ++i) {
            int shift = 3 * q + (2 - i);
            X[i] |= static_cast<uint32_t>((key >> shift) & 1u) << q;
        }
    const uint32_t N = 2u << (bits - 1);
    uint32_t t = X[2] >> 1;
    X[2] ^= X[1];
    X[1] ^= X[0];
    X[0] ^= t;
    for (uint32_t Q = 2; Q != N; Q <<= 1) {
        const uint32_t low = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= low;
            } else {
                uint32_t s = (X[0] ^ X[i]) & low;
                X[0] ^= s;
                X[i] ^= s;
            }
        }
    }
    out[0] = X[0];
    out[1] = X[1];
    out[2] = X[2];
}

// Number of keys of the sorted array P that are < key (std::lower_bound).
uint64_t lower_bound_pos(const uint64_t* P, uint64_t n, uint64_t key) {
    return static_cast<uint64_t>(std::lower_bound(P, P + n, key) - P);
}

// Top-down recursive reference for the balanced leaves (reading R5/R6): a node
// is split iff it holds more than n_crit particles and is above level L.
void split_node(const uint64_t* P, uint64_t n, uint32_t n_crit, uint64_t start, int level,
                std::vector<uint64_t>& K) {
    uint64_t end = start + pow8(kL - level);
    uint64_t count = lower_bound_pos(P, n, end) - lower_bound_pos(P, n, start);
    if (count > n_crit && level < kL) {
        for (uint64_t j = 0; j < 8; ++j) split_node(P, n, n_crit, start + j * pow8(kL - level - 1), level + 1, K);
    } else {
        K.push_back(start);
    }
}


// ---- Node geometry (used by the focus-tree MAC, Sec. 7) --------------------

// Inverse of morton(): bit 3b+2 of the key is bit b of x, 3b+1 of y, 3b of z.
void morton_decode(uint64_t key, uint32_t out[3]) {
    out[0] = out[1] = out[2] = 0;
    for (int b = 0; b < kL; ++b) {
        out[0] |= static_cast<uint32_t>((key >> (3 * b + 2)) & 1u) << b;
        out[1] |= static_cast<uint32_t>((key >> (3 * b + 1)) & 1u) << b;
        out[2] |= static_cast<uint32_t>((key >> (3 * b)) & 1u) << b;
    }
}

// Grid box of the node whose key range starts at `start` on `level`: an
// aligned block of 8^(L - level) keys is an aligned cube of edge
// 2^(L - level) grid cells (Sec. 3), so its lower corner is any of its cells'
// coordinates with the low L - level bits cleared.
void node_box(uint64_t start, int level, int curve, uint32_t lo[3], uint32_t* edge) {
    uint32_t c[3];
    if (curve == 0)
        morton_decode(start, c);
    else
        hilbert_decode(start, kL, c);
    const uint32_t side = 1u << (kL - level);
    for (int d = 0; d < 3; ++d) lo[d] = c[d] & ~(side - 1u);
    *edge = side;
}

// Squared distance between two closed axis-aligned boxes of the grid (0 if
// they touch or overlap), exact in integers.
uint64_t box_dist2(const uint32_t a[3], uint32_t ea, const uint32_t b[3], uint32_t eb) {
    uint64_t r2 = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t gap = 0;
        const int64_t a0 = a[d], a1 = static_cast<int64_t>(a[d]) + ea;
        const int64_t b0 = b[d], b1 = static_cast<int64_t>(b[d]) + eb;
        if (b0 > a1) gap = b0 - a1;
        if (a0 > b1) gap = a0 - b1;
        r2 += static_cast<uint64_t>(gap * gap);
    }
    return r2;
}

// The SFC range [fa, fb) as maximal aligned key blocks (start, level), left to
// right: at each position the largest block 8^e that starts there and ends
// by fb.
std::vector<std::pair<uint64_t, int>> range_blocks(uint64_t fa, uint64_t fb) {
    std::vector<std::pair<uint64_t, int>> out;
    uint64_t k = fa;
    while (k < fb) {
        int e = kL;
        while (e > 0 && (k % pow8(e) != 0 || fb - k < pow8(e))) --e;
        out.push_back({k, kL - e});
        k += pow8(e);
    }
    return out;
}

// Minimum-distance MAC (Sec. 7.1) of the node (start, level) against the focus
// range F = [fa, fb): it fails if some point of F is at distance r_min <= l /
// theta from the node, l the node's edge. In squares: fails iff
// r_min^2 * theta^2 <= l^2, with r_min^2 exact and theta^2 = theta * theta, one
// IEEE double rounding each. With no point in F (fa == fb) it never fails.
bool mac_fails(uint64_t start, int level, int curve, const std::vector<std::pair<uint64_t, int>>& F,
               double theta) {
    uint32_t lo[3], edge;
    node_box(start, level, curve, lo, &edge);
    const double theta2 = theta * theta;
    const double l2 = static_cast<double>(edge) * static_cast<double>(edge);
    for (const auto& blk : F) {
        uint32_t flo[3], fe;
        node_box(blk.first, blk.second, curve, flo, &fe);
        const uint64_t r2 = box_dist2(lo, edge, flo, fe);
        if (!(static_cast<double>(r2) * theta2 > l2)) return true;
    }
    return false;
}

// Top-down reference of the focused tree (Sec. 7.1 definition): a node is
// split iff it holds more than n_crit particles, is above level L and fails
// the MAC against F (every node that overlaps F fails it, r_min being 0).
void split_focus(const uint64_t* P, uint64_t n, uint32_t n_crit, uint64_t start, int level, int curve,
                 const std::vector<std::pair<uint64_t, int>>& F, double theta, std::vector<uint64_t>& K) {
    uint64_t end = start + pow8(kL - level);
    uint64_t count = lower_bound_pos(P, n, end) - lower_bound_pos(P, n, start);
    if (count > n_crit && level < kL && mac_fails(start, level, curve, F, theta)) {
        for (uint64_t j = 0; j < 8; ++j)
            split_focus(P, n, n_crit, start + j * pow8(kL - level - 1), level + 1, curve, F, theta, K);
    } else {
        K.push_back(start);
    }
}

}  // namespace

extern "C" {

// Grid coordinates of each particle (reading R1). Returns 1 if any coordinate
// is NaN or infinite, else 0.
int oracle_quantize(const double* x, const double* y, const double* z, uint64_t n, const double* lo,
                    const double* hi, uint32_t* ix, uint32_t* iy, uint32_t* iz) {
    const double s[3] = {2097152.0 / (hi[0] - lo[0]), 2097152.0 / (hi[1] - lo[1]),
                         2097152.0 / (hi[2] - lo[2])};
    int nonfinite = 0;
    for (uint64_t p = 0; p < n; ++p) {
        if (!std::isfinite(x[p]) || !std::isfinite(y[p]) || !std::isfinite(z[p])) nonfinite = 1;
        ix[p] = quantize_one(x[p], lo[0], s[0]);
        iy[p] = quantize_one(y[p], lo[1], s[1]);
        iz[p] = quantize_one(z[p], lo[2], s[2]);
    }
    return nonfinite;
}

uint64_t oracle_morton_key(uint32_t ix, uint32_t iy, uint32_t iz) { return morton(ix, iy, iz); }

uint64_t oracle_hilbert_key(uint32_t ix, uint32_t iy, uint32_t iz, int bits) { return hilbert(ix, iy, iz, bits); }

void oracle_hilbert_decode(uint64_t key, int bits, uint32_t* out3) { hilbert_decode(key, bits, out3); }

// Sec. 3 + reading R1-R3: SFC key of every particle. curve 0 = Morton,
// 1 = Hilbert. Returns 1 if any coordinate is non-finite.
int oracle_compute_keys(const double* x, const double* y, const double* z, uint64_t n, const double* lo,
                        const double* hi, int curve, uint64_t* keys) {
    std::vector<uint32_t> ix(n), iy(n), iz(n);
    int nonfinite = oracle_quantize(x, y, z, n, lo, hi, ix.data(), iy.data(), iz.data());
    for (uint64_t p = 0; p < n; ++p)
        keys[p] = curve == 0 ? morton(ix[p], iy[p], iz[p]) : hilbert(ix[p], iy[p], iz[p], kL);
    return nonfinite;
}

// Sec. 4 (P is the radix-sorted key array; Table 1: sort_by_key with the
// identity permutation as values). Reading R4: ties keep ascending original
// index, obtained here by sorting (key, index) pairs lexicographically.
void oracle_sort(const uint64_t* keys, uint64_t n, uint64_t* sorted, uint32_t* perm) {
    std::vector<std::pair<uint64_t, uint32_t>> kv(n);
    for (uint64_t p = 0; p < n; ++p) kv[p] = {keys[p], static_cast<uint32_t>(p)};
    std::sort(kv.begin(), kv.end());
    for (uint64_t p = 0; p < n; ++p) {
        sorted[p] = kv[p].first;
        perm[p] = kv[p].second;
    }
}

// Eq. histogram (f): N_i = number of keys of P in [K_i, K_{i+1}), as the
// difference of two binary-search positions.
void oracle_node_counts(const uint64_t* P, uint64_t n, const uint64_t* K, uint64_t n_leaves, uint32_t* counts) {
    for (uint64_t i = 0; i < n_leaves; ++i)
        counts[i] = static_cast<uint32_t>(lower_bound_pos(P, n, K[i + 1]) - lower_bound_pos(P, n, K[i]));
}

// Balanced cornerstone array (Sec. 4) by top-down recursion from the root.
// Writes K (n_l + 1 keys) if it fits in `capacity` keys and returns n_l.
uint64_t oracle_build_leaves(const uint64_t* P, uint64_t n, uint32_t n_crit, uint64_t* K, uint64_t capacity) {
    std::vector<uint64_t> leaves;
    split_node(P, n, n_crit, 0, 0, leaves);
    leaves.push_back(kRootEnd);
    if (leaves.size() <= capacity) std::memcpy(K, leaves.data(), leaves.size() * sizeof(uint64_t));
    return leaves.size() - 1;
}

// One literal application of g = g3 . g2 . g1 (Eqs. g1-g3, rebalancecopy,
// rebalancesplit) to a cornerstone array K with leaf counts N. Writes K' (if
// it fits in `capacity` keys) and its leaf count; returns 1 if some O_i != 1
// (reading R8), else 0.
int oracle_rebalance_step(const uint64_t* K, uint64_t n_leaves, const uint32_t* N, uint32_t n_crit,
                          uint64_t* K_out, uint64_t capacity, uint64_t* n_leaves_out) {
    const uint64_t nl = n_leaves;
    std::vector<uint64_t> O(nl + 1, 0);
    int changed = 0;
    // g1: the rebalance decision for every leaf.
    for (uint64_t i = 0; i < nl; ++i) {
        const uint64_t delta = K[i + 1] - K[i];
        uint64_t op = 1;
        if (N[i] > n_crit && delta > 1) {
            op = 8;  // subdivide (reading R6: a leaf of span 1 cannot be split)
        } else if (delta < kRootEnd) {  // reading R7: the root never merges
            const uint64_t j = (K[i] % (8 * delta)) / delta;  // position among its 7 siblings
            if (j >= 1 && i >= j && i - j + 8 <= nl && K[i - j] + 8 * delta == K[i - j + 8]) {
                uint64_t group = 0;
                for (uint64_t m = 0; m < 8; ++m) group += N[i - j + m];
                if (group <= n_crit) op = 0;  // reading R5: merge iff the 8 counts sum to <= n_crit
            }
        }
        O[i] = op;
        if (op != 1) changed = 1;
    }
    // g2: exclusive prefix sum; O'_{n_l} is the new leaf count.
    std::vector<uint64_t> Op(nl + 1, 0);
    for (uint64_t i = 0; i < nl; ++i) Op[i + 1] = Op[i] + O[i];
    const uint64_t nl_new = Op[nl];
    *n_leaves_out = nl_new;
    if (nl_new + 1 > capacity) return changed;
    // g3: copy or subdivide; reading R10: the closing key 8^L goes last.
    for (uint64_t i = 0; i < nl; ++i) {
        const uint64_t delta = K[i + 1] - K[i];
        if (O[i] == 1) {
            K_out[Op[i]] = K[i];
        } else if (O[i] == 8) {
            for (uint64_t j = 0; j < 8; ++j) K_out[Op[i] + j] = K[i] + j * (delta / 8);
        }
    }
    K_out[nl_new] = kRootEnd;
    return changed;
}

// Number of nodes (internal + leaves) of the fully linked octree over K.
// Sec. 5: n_i = (n_l - 1) / 7.
uint64_t oracle_node_count(uint64_t n_leaves) { return n_leaves + (n_leaves - 1) / 7; }

// Fully linked octree (Sec. 5) by explicit node enumeration: every leaf, plus
// every internal node, emitted once at the leaf where its key range starts.
// Node keys use the placeholder-bit format: a leading 1 followed by the node's
// `level` octal digits. NK is sorted ascending (breadth-first order), LO[l] is
// the first node of level l (reading R15: 23 entries, LO[22] = n), and CO[p]
// is the index of the first child of node p, 0 for leaves. Returns n.
uint64_t oracle_link_octree(const uint64_t* K, uint64_t n_leaves, uint64_t* NK, uint32_t* CO, uint32_t* LO) {
    std::vector<uint64_t> nodes;
    nodes.reserve(oracle_node_count(n_leaves));
    for (uint64_t i = 0; i < n_leaves; ++i) {
        const int leaf_level = level_of_span(K[i + 1] - K[i]);
        for (int l = 0; l <= leaf_level; ++l) {
            // a node of level l < leaf level starts here only if K_i is aligned to its span
            if (l < leaf_level && K[i] % pow8(kL - l) != 0) continue;
            nodes.push_back((1ull << (3 * l)) | (K[i] >> (3 * (kL - l))));
        }
    }
    std::sort(nodes.begin(), nodes.end());
    const uint64_t n = nodes.size();
    std::memcpy(NK, nodes.data(), n * sizeof(uint64_t));
    for (int l = 0; l <= kL; ++l) LO[l] = static_cast<uint32_t>(lower_bound_pos(NK, n, 1ull << (3 * l)));
    LO[kL + 1] = static_cast<uint32_t>(n);
    for (uint64_t p = 0; p < n; ++p) {
        CO[p] = 0;
        if (NK[p] < (1ull << (3 * kL))) {  // nodes on level 21 have no children
            const uint64_t child = NK[p] << 3;
            const uint64_t c = lower_bound_pos(NK, n, child);
            if (c < n && NK[c] == child) CO[p] = static_cast<uint32_t>(c);
        }
    }
    return n;
}

// ---- Node properties (Sec. 5: properties of all n nodes in separate arrays) --

// Particle count of every node of a linked octree (NK in placeholder-bit
// format): the number of keys of P inside the node's key range, i.e. Eq.
// histogram applied to every node, leaves and internal nodes alike.
void oracle_octree_node_counts(const uint64_t* P, uint64_t n, const uint64_t* NK, uint64_t n_nodes,
                               uint32_t* counts) {
    for (uint64_t p = 0; p < n_nodes; ++p) {
        int level = 0;
        while (level < kL && (NK[p] >> (3 * (level + 1))) != 0) ++level;  // the placeholder bit sits at 3 * level
        const uint64_t start = (NK[p] ^ (1ull << (3 * level))) << (3 * (kL - level));
        const uint64_t end = start + pow8(kL - level);
        counts[p] = static_cast<uint32_t>(lower_bound_pos(P, n, end) - lower_bound_pos(P, n, start));
    }
}

// ---- SFC domain decomposition (Sec. 6) ---------------------------------------

// Group the n_l leaves into n_ranks bins of consecutive leaves holding about
// N / n_ranks particles each. With C_i the number of particles in leaves
// before leaf i (C_0 = 0, C_{n_l} = N), bin r starts at the first leaf
// boundary at or past r N / n_ranks: bounds[r] = min { i : C_i * n_ranks >=
// r * N }, so bounds[0] = 0 and bounds[n_ranks] = n_l (exact integers).
void oracle_sfc_partition(const uint32_t* counts, uint64_t n_leaves, uint32_t n_ranks, uint32_t* bounds) {
    std::vector<uint64_t> C(n_leaves + 1, 0);
    for (uint64_t i = 0; i < n_leaves; ++i) C[i + 1] = C[i] + counts[i];
    const uint64_t N = C[n_leaves];
    for (uint32_t r = 0; r <= n_ranks; ++r) {
        uint64_t i = 0;
        while (i < n_leaves && C[i] * n_ranks < static_cast<uint64_t>(r) * N) ++i;
        bounds[r] = static_cast<uint32_t>(r == n_ranks ? n_leaves : i);
    }
}

// ---- Focused (locally essential) tree on one GPU's data (Sec. 7) --------------

// Minimum-distance MAC of one node against the focus range [fa, fb); returns
// 1 if it fails (the node must be resolved further for F), else 0.
int oracle_mac_fails(uint64_t start, int level, int curve, uint64_t fa, uint64_t fb, double theta) {
    return mac_fails(start, level, curve, range_blocks(fa, fb), theta) ? 1 : 0;
}

// Grid box (lower corner and edge) of the node (start, level).
void oracle_node_box(uint64_t start, int level, int curve, uint32_t* lo3, uint32_t* edge) {
    node_box(start, level, curve, lo3, edge);
}

// The focused cornerstone array by top-down recursion (split iff count >
// n_crit, level < L and the MAC fails). Writes K if it fits in `capacity`
// keys; returns n_l.
uint64_t oracle_focus_leaves(const uint64_t* P, uint64_t n, uint32_t n_crit, int curve, uint64_t fa, uint64_t fb,
                             double theta, uint64_t* K, uint64_t capacity) {
    std::vector<uint64_t> leaves;
    split_focus(P, n, n_crit, 0, 0, curve, range_blocks(fa, fb), theta, leaves);
    leaves.push_back(kRootEnd);
    if (leaves.size() <= capacity) std::memcpy(K, leaves.data(), leaves.size() * sizeof(uint64_t));
    return leaves.size() - 1;
}

// One literal update g^LE = g3 . g2 . g^LE_1 (Sec. 7.2) of the focused array K
// with leaf counts N. g^LE_1: split a leaf if it holds more than n_crit
// particles, can be split and fails the MAC; merge a complete group of 8
// sibling leaves if their parent holds at most n_crit particles or passes the
// MAC; otherwise keep. Inside F (and wherever a node overlaps F) the MAC always
// fails, so the rule there is g1's. Returns 1 if some O_i != 1.
int oracle_focus_rebalance_step(const uint64_t* K, uint64_t n_leaves, const uint32_t* N, uint32_t n_crit, int curve,
                                uint64_t fa, uint64_t fb, double theta, uint64_t* K_out, uint64_t capacity,
                                uint64_t* n_leaves_out) {
    const uint64_t nl = n_leaves;
    const auto F = range_blocks(fa, fb);
    std::vector<uint64_t> O(nl + 1, 0);
    int changed = 0;
    for (uint64_t i = 0; i < nl; ++i) {
        const uint64_t delta = K[i + 1] - K[i];
        const int level = level_of_span(delta);
        uint64_t op = 1;
        if (N[i] > n_crit && delta > 1 && mac_fails(K[i], level, curve, F, theta)) {
            op = 8;
        } else if (delta < kRootEnd) {  // reading R7: the root never merges
            const uint64_t j = (K[i] % (8 * delta)) / delta;
            if (j >= 1 && i >= j && i - j + 8 <= nl && K[i - j] + 8 * delta == K[i - j + 8]) {
                uint64_t group = 0;
                for (uint64_t m = 0; m < 8; ++m) group += N[i - j + m];
                // reading R5 for "smaller than N_crit": the parent's count <= n_crit
                if (group <= n_crit || !mac_fails(K[i - j], level - 1, curve, F, theta)) op = 0;
            }
        }
        O[i] = op;
        if (op != 1) changed = 1;
    }
    std::vector<uint64_t> Op(nl + 1, 0);
    for (uint64_t i = 0; i < nl; ++i) Op[i + 1] = Op[i] + O[i];
    const uint64_t nl_new = Op[nl];
    *n_leaves_out = nl_new;
    if (nl_new + 1 > capacity) return changed;
    for (uint64_t i = 0; i < nl; ++i) {
        const uint64_t delta = K[i + 1] - K[i];
        if (O[i] == 1) {
            K_out[Op[i]] = K[i];
        } else if (O[i] == 8) {
            for (uint64_t j = 0; j < 8; ++j) K_out[Op[i] + j] = K[i] + j * (delta / 8);
        }
    }
    K_out[nl_new] = kRootEnd;
    return changed;
}

// ---- Binary radix tree over sorted unique keys (Sec. 5, after Karras) --------

// For m sorted unique keys k_0 < ... < k_{m-1} (63-bit), the binary radix tree
// has one internal node per adjacent pair (i, i + 1): the node whose key
// ranges split between them. Its prefix is the common prefix of k_i and
// k_{i+1}, of prefix_len[i] = (leading zeros of k_i XOR k_{i+1}) - 1 bits
// within the 63-bit key (reading R11). Its key range [first[i], last[i]] is
// the maximal run of keys sharing that prefix. Found here by scanning outwards
// from the pair, one key at a time.
void oracle_radix_nodes(const uint64_t* k, uint64_t m, uint32_t* prefix_len, uint32_t* first, uint32_t* last) {
    for (uint64_t i = 0; i + 1 < m; ++i) {
        const int d = __builtin_clzll(k[i] ^ k[i + 1]) - 1;
        prefix_len[i] = static_cast<uint32_t>(d);
        const uint64_t pre = k[i] >> (63 - d);
        uint64_t a = i, b = i + 1;
        while (a > 0 && (k[a - 1] >> (63 - d)) == pre) --a;
        while (b + 1 < m && (k[b + 1] >> (63 - d)) == pre) ++b;
        first[i] = static_cast<uint32_t>(a);
        last[i] = static_cast<uint32_t>(b);
    }
}

// Compact octree (Sec. 5, the binary radix tree with the empty buckets of K
// removed): the leaves of K that hold particles, plus one internal node for
// every node of the binary radix tree over those leaves' keys whose prefix
// length is a multiple of 3 (each adjacent pair of leaf keys splits exactly
// one binary node, of prefix length = their common prefix), plus the root
// (reading: the whole domain is always a node, so that the nodes form one
// tree even where the radix tree's top prefix is not a whole digit). Node
// keys in placeholder-bit format, sorted (breadth-first order); parent[p] is
// the index of the nearest proper ancestor present (its longest proper prefix
// among the nodes), 0xffffffff for the root. Writes up to `capacity` nodes
// and returns their number.
uint64_t oracle_compact_octree(const uint64_t* K, uint64_t n_leaves, const uint32_t* counts, uint64_t* NK,
                               uint32_t* parent, uint64_t capacity) {
    std::vector<uint64_t> keys, leaf_nodes;
    for (uint64_t i = 0; i < n_leaves; ++i) {
        if (counts[i] == 0) continue;
        const int level = level_of_span(K[i + 1] - K[i]);
        keys.push_back(K[i]);
        leaf_nodes.push_back((1ull << (3 * level)) | (K[i] >> (3 * (kL - level))));
    }
    std::vector<uint64_t> nodes = leaf_nodes;
    for (size_t i = 0; i + 1 < keys.size(); ++i) {
        const int d = __builtin_clzll(keys[i] ^ keys[i + 1]) - 1;
        if (d % 3 == 0) nodes.push_back((1ull << d) | (d ? keys[i] >> (63 - d) : 0ull));
    }
    if (std::find(nodes.begin(), nodes.end(), 1ull) == nodes.end()) nodes.push_back(1ull);  // the root
    std::sort(nodes.begin(), nodes.end());
    const uint64_t n = nodes.size();
    if (n <= capacity) {
        for (uint64_t p = 0; p < n; ++p) {
            NK[p] = nodes[p];
            parent[p] = 0xffffffffu;
            int level = 0;
            while ((nodes[p] >> (3 * (level + 1))) != 0) ++level;
            for (int up = level - 1; up >= 0; --up) {  // nearest ancestor present
                const uint64_t a = nodes[p] >> (3 * (level - up));
                const uint64_t at = lower_bound_pos(nodes.data(), n, a);
                if (at < n && nodes[at] == a) {
                    parent[p] = static_cast<uint32_t>(at);
                    break;
                }
            }
        }
    }
    return n;
}

// Convenience: the whole pipeline of Secs. 3-5 for one particle set.
// Returns n_l; K must hold up to `leaf_capacity` + 1 keys. If n_l exceeds the
// capacity nothing past the keys and the sort is written.
uint64_t oracle_build(const double* x, const double* y, const double* z, uint64_t n, const double* lo,
                      const double* hi, int curve, uint32_t n_crit, uint64_t* sorted_keys, uint32_t* perm,
                      uint64_t* K, uint64_t leaf_capacity, uint32_t* counts) {
    std::vector<uint64_t> keys(n);
    oracle_compute_keys(x, y, z, n, lo, hi, curve, keys.data());
    oracle_sort(keys.data(), n, sorted_keys, perm);
    uint64_t nl = oracle_build_leaves(sorted_keys, n, n_crit, K, leaf_capacity + 1);
    if (nl <= leaf_capacity) oracle_node_counts(sorted_keys, n, K, nl, counts);
    return nl;
}

}  // extern "C"
