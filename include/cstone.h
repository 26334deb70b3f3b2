/*
 * cstone.h — C ABI of the MI355X (gfx950) Cornerstone octree build.
 *
 * Implements the single-GPU octree construction of Keller et al.,
 * "Cornerstone: Octree Construction Algorithms for Scalable Particle
 * Simulations" (PASC '23): SFC keys (Sec. 3), the sorted key array P with its
 * particle permutation (Sec. 4, Table 1), leaf counts f (Eq. histogram), the
 * iterated rebalance g = g3.g2.g1 (Eqs. g1-g3, rebalancecopy, rebalancesplit)
 * and the fully linked octree NK / CO / LO (Sec. 5).
 *
 * Conventions shared by every call
 *   - L = 21: keys are uint64 in [0, 8^21) = [0, 2^63); 8^21 = 2^63 closes every
 *     cornerstone array (Eq. cstone). Counts, permutation, CO and LO are uint32,
 *     so n < 2^32.
 *   - All array pointers are DEVICE pointers owned by the caller unless marked
 *     "host". The library keeps no pointer after a call returns and never
 *     allocates device memory: scratch comes from the caller's workspace `ws`,
 *     sized by the matching *_workspace_bytes() query (any 256-byte aligned
 *     device buffer of at least that size; its contents on entry do not matter).
 *   - Every call enqueues its work on `stream`. Calls that return results on the
 *     host (cstone_rebalance, cstone_build) synchronise `stream` before
 *     returning; the others are asynchronous.
 *   - Functions return a cstone_status and never abort. Output arrays are
 *     unspecified after an error unless stated otherwise.
 *   - Overlapping calls that share one workspace race; give concurrent calls on
 *     different streams their own workspaces.
 */
#ifndef CSTONE_H
#define CSTONE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Every entry point below is exported from libcstone.so; nothing else is. */
#define CSTONE_API __attribute__((visibility("default")))

typedef enum cstone_status {
    CSTONE_OK = 0,
    CSTONE_ERR_INVALID_ARG = 1,   /* null pointer, n >= 2^32, n_crit == 0, bad box, short workspace */
    CSTONE_ERR_NONFINITE = 2,     /* a coordinate is NaN or infinite */
    CSTONE_ERR_CAPACITY = 3,      /* the next cornerstone array would exceed leaf_capacity */
    CSTONE_ERR_NOT_CONVERGED = 4, /* max_iters rounds ran and some leaf still changed */
    CSTONE_ERR_DEVICE = 5,        /* a HIP runtime error, or a device-side wait gave up */
} cstone_status;

typedef enum cstone_curve {
    CSTONE_MORTON = 0,  /* Morton Z-curve; x is the most significant bit of each octal digit */
    CSTONE_HILBERT = 1, /* Skilling's 3D Hilbert curve, x most significant; key 0 at the origin */
} cstone_curve;

/* Axis-aligned bounding box (host struct): lo[d] < hi[d], all finite. */
typedef struct cstone_box {
    double lo[3];
    double hi[3];
} cstone_box;

/* Bit OR-ed into the optional device flag word of cstone_compute_keys. */
#define CSTONE_FLAG_NONFINITE 1u

/* Number of entries of the level-offset array LO (Sec. 5: L + 2). */
#define CSTONE_LEVEL_OFFSETS 23

/* Human-readable name of a status code (static string). */
CSTONE_API const char* cstone_status_string(cstone_status status);

/* ------------------------------------------------------------------------
 * Keys (Sec. 3). For every particle p, the coordinates are mapped to the
 * integer grid [0, 2^21)^3 by t = (c - lo) * (2^21 / (hi - lo)) in IEEE double
 * (one rounding per operation, no contraction), clamped to [0, 2^21 - 1] and
 * truncated; NaN maps to 0 and +Inf to 2^21 - 1. The grid point is encoded on
 * the chosen curve into keys[p].
 *   x, y, z   device, n doubles each (structure of arrays)
 *   box       host, bounding box
 *   keys      device, n uint64 (output)
 *   flags     device, one uint32 or NULL; CSTONE_FLAG_NONFINITE is OR-ed in if
 *             any coordinate is NaN or infinite (the word is not cleared).
 * Asynchronous. Errors: INVALID_ARG, DEVICE.
 */
CSTONE_API cstone_status cstone_compute_keys(const double* x, const double* y, const double* z, size_t n,
                                  const cstone_box* box, cstone_curve curve, uint64_t* keys,
                                  uint32_t* flags, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Sort (Sec. 4, Table 1: radix sort_by_key with the identity permutation as
 * values). Stable radix sort: keys_out[i] = keys_in[perm_out[i]], keys_out
 * non-decreasing, equal keys in ascending original index. Keys are particle
 * keys: 63 significant bits (bit 63 is not sorted on). Three digit passes
 * order the keys by their top 27 bits; the runs of one 27-bit prefix are then
 * sorted in place, in LDS, or by four passes over their low 36 bits if longer
 * than 2048 keys.
 *   keys_in   device, n uint64 below 2^63 (not modified; may not alias the outputs)
 *   keys_out  device, n uint64;  perm_out  device, n uint32
 *   ws        device workspace of cstone_sort_workspace_bytes(n) bytes
 * Asynchronous. Errors: INVALID_ARG, DEVICE.
 */
CSTONE_API size_t cstone_sort_workspace_bytes(size_t n);
CSTONE_API cstone_status cstone_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Leaf counts f (Eq. histogram): counts[i] = number of keys of the sorted array
 * in [leaves[i], leaves[i+1]), as the difference of two binary-search
 * positions.
 *   sorted_keys  device, n uint64, non-decreasing
 *   leaves       device, n_leaves + 1 uint64, a cornerstone array
 *   counts       device, n_leaves uint32 (output)
 * Asynchronous. Errors: INVALID_ARG, DEVICE.
 */
CSTONE_API cstone_status cstone_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves,
                                 size_t n_leaves, uint32_t* counts, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Rebalance loop (Sec. 4): alternate f and g = g3.g2.g1 until no leaf is
 * split or merged (O_i = 1 for all i), starting from the cornerstone array in
 * `leaves`. A leaf splits if it holds more than n_crit particles and spans
 * more than one key; 8 sibling leaves merge if their counts sum to at most
 * n_crit; the root never merges. From the single root leaf {0, 8^21} the result
 * is the unique balanced array (leaf counts <= n_crit, internal node counts >
 * n_crit).
 *   sorted_keys  device, n uint64, non-decreasing
 *   leaves       device, leaf_capacity + 1 uint64; in: the start array (a
 *                previous step's result; with *n_leaves == 1 the root array
 *                {0, 2^63} is written here), out: the final array
 *   n_leaves     host, in: leaves in the start array (>= 1), out: final count
 *                (on CAPACITY: the count the next round needed)
 *   counts       device, leaf_capacity uint32 (output: final leaf counts), or NULL
 *   max_iters    rounds allowed (0 means 22 = L + 1)
 *   iters_done   host, rounds run (a round is one f + one g), or NULL
 *   ws           device workspace of cstone_rebalance_workspace_bytes(n, n_crit,
 *                leaf_capacity) bytes
 * Synchronises `stream`. Errors: INVALID_ARG; CAPACITY (leaves keep the last
 * array that fitted, *n_leaves is the count the next round needed);
 * NOT_CONVERGED (leaves hold the array after max_iters rounds, a valid
 * cornerstone array); DEVICE.
 */
CSTONE_API size_t cstone_rebalance_workspace_bytes(size_t n, uint32_t n_crit, size_t leaf_capacity);
CSTONE_API cstone_status cstone_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves,
                               size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                               uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* Leaf capacity that a rebalance of n particles can never exceed: every round
 * from the root only splits, and a balanced tree has at most
 * floor(n / (n_crit + 1)) internal nodes per level, so 7 * 21 * that + 1;
 * starting from an array of n_leaves_start leaves, one round adds at most 7 per
 * over-full leaf on top of it. */
CSTONE_API size_t cstone_leaf_capacity_bound(size_t n, uint32_t n_crit, size_t n_leaves_start);

/* ------------------------------------------------------------------------
 * Fully linked octree (Sec. 5). n = n_leaves + (n_leaves - 1) / 7 nodes.
 * Every node is started by one leaf (its first); the nodes of one level are
 * in leaf order, so each node's breadth-first index is a per-level count over
 * the leaves, found by one counting pass, a scan and one writing pass.
 *   node_keys      device, n uint64: every node in Warren-Salmon placeholder-bit
 *                  form (a 1 bit followed by the node's level octal digits),
 *                  ascending = breadth-first (level-major, SFC order within a level)
 *   child          device, n uint32: index of the first of the node's 8
 *                  contiguous children, 0 for a leaf (CO)
 *   level_offsets  device, 23 uint32: index of the first node of each level
 *                  0..21, then n (LO)
 *   ws             device workspace of cstone_link_workspace_bytes(n_leaves) bytes
 * Asynchronous. Errors: INVALID_ARG, DEVICE.
 */
CSTONE_API size_t cstone_node_count(size_t n_leaves);
CSTONE_API size_t cstone_link_workspace_bytes(size_t n_leaves);
CSTONE_API cstone_status cstone_link_octree(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                 uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);

/* Same outputs as cstone_link_octree, computed by the five steps of Sec. 5 as
 * written: leaf and internal node keys (internal nodes at the slot given by
 * Eq. digitweight, with the digit weights' sign reversed so the slots are the
 * integers 0..n_i-1), a radix sort of NK, LO and CO by binary search. Kept for
 * comparison; cstone_link_octree reaches the breadth-first order directly. */
CSTONE_API cstone_status cstone_link_octree_by_sort(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys,
                                                    uint32_t* child, uint32_t* level_offsets, void* ws,
                                                    size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Whole build: keys -> sort -> rebalance loop -> link, on one stream.
 *   x, y, z, box, curve      as cstone_compute_keys
 *   n_crit                   maximum particles per leaf (>= 1)
 *   sorted_keys, perm        device, n each: P and the particle permutation
 *   leaves, n_leaves, leaf_capacity, counts, max_iters, iters_done
 *                            as cstone_rebalance; *n_leaves == 0 on entry means
 *                            "start from the root leaf", otherwise `leaves`
 *                            holds the previous cornerstone array to start from
 *   node_keys, child         device, cstone_node_count(leaf_capacity) entries each,
 *                            or both NULL to skip linking
 *   level_offsets            device, 23 uint32 (ignored when node_keys is NULL)
 *   ws                       device workspace, cstone_build_workspace_bytes(n, leaf_capacity)
 *   timings                  host, or NULL: HIP-event times of the stages and of
 *                            the parts of the particle-key sort (events
 *                            are recorded on `stream` only when this is non-NULL)
 * Synchronises `stream`. Errors: those of the stages; NONFINITE if a
 * coordinate is NaN or infinite (found at the first synchronisation, the
 * outputs are then unspecified and no linking is done).
 */
typedef struct cstone_timings {
    float stage_ms[4];     /* keys, sort, rebalance loop, link */
    float sort_pass_ms[8]; /* the particle-key sort (4 entries): the first top
                              pass, the two later top passes together, the
                              bucket pass, the low passes */
    uint32_t sort_passes;  /* entries of sort_pass_ms in use */
} cstone_timings;

CSTONE_API size_t cstone_build_workspace_bytes(size_t n, size_t leaf_capacity);
CSTONE_API cstone_status cstone_build(const double* x, const double* y, const double* z, size_t n, const cstone_box* box,
                           cstone_curve curve, uint32_t n_crit, uint64_t* sorted_keys, uint32_t* perm,
                           uint64_t* leaves, size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                           uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets, uint32_t max_iters,
                           uint32_t* iters_done, void* ws, size_t ws_bytes, cstone_timings* timings,
                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * cstone_build without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid allocation). Same arguments, outputs and errors as cstone_build,
 * less ws, ws_bytes and timings: the workspace is a fixed device array of
 * CSTONE_STATIC_SCRATCH_BYTES inside the library, held on every device the
 * library runs on until the process ends. Its address on a device is looked up
 * on the first call there. The call allocates nothing.
 * INVALID_ARG if cstone_build_workspace_bytes(n, leaf_capacity) exceeds the
 * array (e.g. n above about 2^21 with a leaf capacity of about 8 n / N_crit);
 * DEVICE if the array cannot be found. Every call on a device shares that
 * device's array, which keeps the last call's contents: calls that overlap on
 * one device (other streams, other host threads) race, so the caller must
 * order them. Synchronises `stream`, as cstone_build does.
 */
#define CSTONE_STATIC_SCRATCH_BYTES (64ull << 20)
CSTONE_API cstone_status cstone_build_static(const double* x, const double* y, const double* z, size_t n,
                                             const cstone_box* box, cstone_curve curve, uint32_t n_crit,
                                             uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                             size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                             uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                             uint32_t max_iters, uint32_t* iters_done, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Octrees by way of a binary radix tree (Sec. 5, after Karras).
 *
 * cstone_radix_tree: the binary radix tree over m sorted unique keys (device,
 * uint64 < 2^63): m - 1 internal nodes, node i covering keys [first[i],
 * last[i]] (one end is i), split after key split[i] (left child: key split[i]
 * if first[i] == split[i], else internal node split[i]; right child: key
 * split[i] + 1 if that is last[i], else internal node split[i] + 1), and
 * prefix_len[i] = the bits its keys share within the 63-bit key; node 0 is
 * the root. Outputs: device, m - 1 uint32 each; first, last and split may be
 * NULL. Asynchronous. Errors: INVALID_ARG.
 *
 * cstone_link_octree_radix: the linked octree of a cornerstone array through
 * the radix tree over its leaf keys: its nodes with a prefix length that is a
 * multiple of 3 are the internal octree nodes, extracted by a flag per node
 * and an exclusive scan, then sorted and linked as in steps 3-5. Outputs
 * equal those of cstone_link_octree. ws:
 * cstone_link_octree_radix_workspace_bytes(n_leaves). Asynchronous.
 *
 * cstone_compact_octree: the octree with the empty buckets of K removed: the
 * leaves whose count is not 0, the internal nodes of the radix tree over their
 * keys whose prefix length is a multiple of 3, and the root (always present,
 * so that the nodes form one tree). Every internal node but the root has at
 * least 2 children. node_keys (device, capacity 2 n_leaves + 1 uint64):
 * placeholder-bit keys in breadth-first order; parent (device, same
 * capacity, uint32): index of the nearest proper ancestor present,
 * 0xffffffff for the root; level_offsets (device, 23 uint32) as LO; *n_nodes
 * (host): the node count. counts: device, n_leaves uint32 (Eq. histogram).
 * Synchronises `stream`. ws: cstone_compact_octree_workspace_bytes(n_leaves).
 */
CSTONE_API cstone_status cstone_radix_tree(const uint64_t* keys, size_t m, uint32_t* first, uint32_t* last,
                                           uint32_t* split, uint32_t* prefix_len, hipStream_t stream);
CSTONE_API size_t cstone_link_octree_radix_workspace_bytes(size_t n_leaves);
CSTONE_API cstone_status cstone_link_octree_radix(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys,
                                                  uint32_t* child, uint32_t* level_offsets, void* ws, size_t ws_bytes,
                                                  hipStream_t stream);
CSTONE_API size_t cstone_compact_octree_workspace_bytes(size_t n_leaves);
CSTONE_API cstone_status cstone_compact_octree(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                               uint64_t* node_keys, uint32_t* parent, uint32_t* level_offsets,
                                               size_t* n_nodes, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Node properties and particles in curve order (Sec. 5: properties of the n
 * nodes kept in separate arrays of length n, filled after the build; Sec. 4:
 * the permutation that sorts the keys, applied to the particle arrays).
 *
 * cstone_octree_node_counts: the particle count of every node of a linked
 * octree, node_counts[p] = number of particles whose key lies in node p's key
 * range. Leaves get their leaf count; an internal node the sum over its
 * children, i.e. what an upward pass over the tree gives (the root holds
 * the sum of all leaf counts).
 *   leaves      device, n_leaves + 1 uint64, the cornerstone array K
 *   counts      device, n_leaves uint32, its leaf counts (Eq. histogram)
 *   node_keys   device, n_nodes uint64, NK of cstone_link_octree on K
 *   node_counts device, n_nodes uint32 (output, same order as node_keys)
 *   ws          device, cstone_octree_node_counts_workspace_bytes(n_leaves)
 * Asynchronous. A node key that does not start at a leaf boundary of K (NK
 * of another tree) gets 0xffffffff. Errors: INVALID_ARG.
 *
 * cstone_gather: dst[i] = src[perm[i]] for i < n (src, dst: device, n
 * doubles, not aliasing; perm: device, a permutation of 0 .. n-1, e.g. from
 * cstone_sort). cstone_gather_xyz does it for x, y, z: as three passes (one
 * array's reads stay in the last-level cache for n up to 2^25) or, with
 * fused != 0, one pass over all three. Asynchronous. Errors: INVALID_ARG.
 */
CSTONE_API size_t cstone_octree_node_counts_workspace_bytes(size_t n_leaves);
CSTONE_API cstone_status cstone_octree_node_counts(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                                   const uint64_t* node_keys, size_t n_nodes, uint32_t* node_counts,
                                                   void* ws, size_t ws_bytes, hipStream_t stream);
CSTONE_API cstone_status cstone_gather(const double* src, const uint32_t* perm, size_t n, double* dst,
                                       hipStream_t stream);
CSTONE_API cstone_status cstone_gather_xyz(const double* x, const double* y, const double* z, const uint32_t* perm,
                                           size_t n, double* ox, double* oy, double* oz, int fused,
                                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * The replicated tree of particles held by several ranks, and the domain
 * decomposition built on it (Sec. 6), for n_shards shards on one device.
 *
 * Shard g holds the particles [shard_offsets[g], shard_offsets[g+1]) (host
 * array, n_shards + 1 entries, non-decreasing from 0 to n). Every round
 * applies f (Eq. histogram) to each shard's own sorted keys, sums the
 * n_shards count arrays element by element (f_r: the global reduction of the
 * counts; a collective across ranks, here a reduction kernel), and applies g
 * (Eqs. g1-g3) to the summed counts, until no leaf changes (f_glob = f_r . f
 * alternating with g). The result is the balanced tree of all particles.
 *
 * cstone_global_rebalance: sorted_keys (device, n uint64) holds each shard's
 * keys sorted on their own, back to back. leaves / n_leaves / leaf_capacity /
 * counts (the summed counts of the final array) / max_iters / iters_done as
 * in cstone_rebalance, and so are its errors. Synchronises `stream` once per
 * round. ws: cstone_global_rebalance_workspace_bytes(leaf_capacity, n_shards).
 *
 * cstone_build_sharded: keys of every particle (Sec. 3), every shard sorted
 * on its own (sorted_keys and perm per shard, perm relative to the shard's
 * first particle), then cstone_global_rebalance from `leaves` (e.g. the root
 * {0, 8^L}). ws: cstone_build_sharded_workspace_bytes (0 for bad offsets).
 * Errors as cstone_build (no linking: cstone_link_octree on the result).
 *
 * cstone_sfc_partition: groups the leaves into n_ranks bins of consecutive
 * leaves holding about N / n_ranks particles each (N the sum of counts):
 * bounds (device, n_ranks + 1 uint32) with bin r = leaves [bounds[r],
 * bounds[r+1]); with C_i the particles in leaves before leaf i, bounds[r] is
 * the least i with C_i * n_ranks >= r * N, and bounds[n_ranks] = n_leaves.
 * Bin r covers the keys [leaves[bounds[r]], leaves[bounds[r+1]]). counts:
 * device, n_leaves uint32. Asynchronous. ws:
 * cstone_sfc_partition_workspace_bytes(n_leaves). Errors: INVALID_ARG.
 */
CSTONE_API size_t cstone_global_rebalance_workspace_bytes(size_t leaf_capacity, uint32_t n_shards);
CSTONE_API cstone_status cstone_global_rebalance(const uint64_t* sorted_keys, const uint64_t* shard_offsets,
                                                 uint32_t n_shards, uint32_t n_crit, uint64_t* leaves,
                                                 size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                                 uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                                 hipStream_t stream);
CSTONE_API size_t cstone_build_sharded_workspace_bytes(const uint64_t* shard_offsets, uint32_t n_shards,
                                                       size_t leaf_capacity);
CSTONE_API cstone_status cstone_build_sharded(const double* x, const double* y, const double* z,
                                              const uint64_t* shard_offsets, uint32_t n_shards,
                                              const cstone_box* box, cstone_curve curve, uint32_t n_crit,
                                              uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                              size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                              uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                              hipStream_t stream);
CSTONE_API size_t cstone_sfc_partition_workspace_bytes(size_t n_leaves);
CSTONE_API cstone_status cstone_sfc_partition(const uint32_t* counts, size_t n_leaves, uint32_t n_ranks,
                                              uint32_t* bounds, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The tree focused on a range of the curve (Sec. 7: a locally essential tree
 * for the subdomain F = [focus_start, focus_end) of one rank), from the
 * particles at hand (the counts need no communication here).
 *
 * Minimum-distance MAC (Sec. 7.1): a node of edge l fails it against F if
 * some point of F lies within distance l / theta of the node; distances are
 * measured in grid cells between the closed grid boxes of the node and of F
 * (F cut into maximal aligned key blocks), as r^2 theta^2 <= l^2 with r^2
 * exact and theta^2 = theta * theta. A node overlapping F always fails;
 * theta = 0 makes every node fail; an empty F makes none fail.
 *
 * cstone_focus_rebalance: rounds of f (Eq. histogram) and g^LE = g3 . g2 .
 * g^LE_1 (Sec. 7.2) until no leaf changes, from `leaves` (e.g. the root).
 * g^LE_1 splits a leaf holding more than n_crit particles only if it fails
 * the MAC, and merges a complete group of 8 sibling leaves if their parent
 * holds at most n_crit particles or passes the MAC; inside F this is g1. The
 * result is the unique tree in which a node is split iff it holds more than
 * n_crit particles, lies above level L and fails the MAC. Arguments, outputs
 * and errors as cstone_rebalance; theta >= 0 and finite, focus_start <=
 * focus_end <= 8^L. Synchronises `stream` once per round.
 * ws: cstone_focus_rebalance_workspace_bytes(leaf_capacity).
 *
 * cstone_focus_mac (f^LE_2): fails[p] = 1 if node p of a linked octree (NK,
 * placeholder-bit keys, device, n_nodes uint64) fails the MAC against F, else
 * 0 (device, n_nodes bytes). Asynchronous.
 * ws: cstone_focus_mac_workspace_bytes().
 */
CSTONE_API size_t cstone_focus_rebalance_workspace_bytes(size_t leaf_capacity);
CSTONE_API cstone_status cstone_focus_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit,
                                                cstone_curve curve, uint64_t focus_start, uint64_t focus_end,
                                                double theta, uint64_t* leaves, size_t* n_leaves,
                                                size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                                                uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream);
CSTONE_API size_t cstone_focus_mac_workspace_bytes(void);
CSTONE_API cstone_status cstone_focus_mac(const uint64_t* node_keys, size_t n_nodes, cstone_curve curve,
                                          uint64_t focus_start, uint64_t focus_end, double theta, uint8_t* fails,
                                          void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Sort tile shapes and their autotune table. The radix sort has several
 * compiled shapes (digit width, block size, keys per thread). Which one a
 * sort runs is looked up once, when the sort (or build) starts, in a
 * process-wide table keyed by (kernel, size class, device):
 *   kernel      CSTONE_TUNE_SORT: the particle-key sort of cstone_sort and
 *               cstone_build; CSTONE_TUNE_BATCH_SORT: the segmented sort of a
 *               batch plan (looked up by cstone_batch_create, n = all its
 *               particles);
 *   size class  floor(log2 n);
 *   device      the current HIP device's architecture and compute-unit count.
 * Without an entry the built-in shape (index 0) is used. Every shape gives
 * the same result (the sort is stable), so the table changes speed only.
 * The table is the library's only process-wide state; its calls are
 * thread-safe, and a sort already started keeps the shape it looked up.
 *   cstone_sort_autotune  sorts keys_in (device, n, < 2^63) with every shape,
 *                         reps times each after a warm-up, writes the mean
 *                         times (host, one per shape, or NULL) and the index
 *                         chosen, and records it for (CSTONE_TUNE_SORT, n,
 *                         this device). ws: cstone_sort_workspace_bytes(n).
 *                         Synchronises `stream`.
 *   cstone_tune_set       records `variant` for (kernel, size class of n, this
 *                         device); -1 removes that entry. INVALID_ARG for an
 *                         unknown kernel or shape.
 *   cstone_tune_get       the recorded shape for (kernel, n, this device), or -1.
 *   cstone_tune_clear     empties the table; cstone_tune_entries counts it.
 *   cstone_tune_save      writes the table to a JSON file (one entry per line:
 *                         kernel, size_log2, device, variant and the shape's
 *                         digit bits, block, items and split).
 *                         INVALID_ARG if the file cannot be written.
 *   cstone_tune_load      merges such a file into the table, skipping entries
 *                         whose index does not name the same shape in this
 *                         library. INVALID_ARG if the file cannot be read or
 *                         is not in that format (the table is then unchanged).
 */
#define CSTONE_TUNE_SORT 0
#define CSTONE_TUNE_BATCH_SORT 1
CSTONE_API int cstone_sort_variant_count(void);
CSTONE_API cstone_status cstone_sort_variant_info(int variant, int* digit_bits, int* block, int* items);
/* The rest of a shape: whether particle keys take the split sort (1) or
 * plain LSD passes (0). */
CSTONE_API cstone_status cstone_sort_variant_split(int variant, int* split);
/* Look-back waits before a sort block counts a missing predecessor tile's
 * digits itself (the look-back's fallback), for later launches on the current
 * device; default 256. Any value gives the same sort; 0 sends every wait to
 * the fallback (for tests). Errors: DEVICE. */
CSTONE_API cstone_status cstone_set_lookback_patience(uint32_t waits);
CSTONE_API cstone_status cstone_sort_autotune(const uint64_t* keys_in, size_t n, uint64_t* keys_out, uint32_t* perm_out,
                                   void* ws, size_t ws_bytes, int reps, float* ms_per_variant, int* chosen,
                                   hipStream_t stream);
CSTONE_API cstone_status cstone_tune_set(int kernel, size_t n, int variant);
CSTONE_API int cstone_tune_get(int kernel, size_t n);
CSTONE_API void cstone_tune_clear(void);
CSTONE_API size_t cstone_tune_entries(void);
CSTONE_API cstone_status cstone_tune_save(const char* path);
CSTONE_API cstone_status cstone_tune_load(const char* path);

/* ------------------------------------------------------------------------
 * Batched builds: many independent particle sets (Sec. 4-5 for each), of
 * uneven sizes and N_crit, built from their root leaves by one sequence of
 * launches with no host synchronisation (every stage is a single launch over
 * all sets: per-tile set tables for the keys and the segmented sort, the sets'
 * cornerstone arrays kept back to back through the rebalance rounds with one
 * scan per round and per-set convergence flags, one linking pass). The
 * sequence can be captured once into a hipGraph and replayed. With a 9-bit
 * sort shape the segmented sort is the split sort of cstone_sort applied per
 * set (every set's first key starts a bucket); 8-bit shapes take LSD passes.
 * Both are stable, so the results do not depend on the shape.
 *
 * Layout. Particles of set s occupy [particle_offsets[s], particle_offsets[s+1])
 * of x, y, z, sorted_keys and perm (perm values count from the set's first
 * particle). Its cornerstone array goes to leaves[leaf_offsets[s] ...] (n_leaves
 * + 1 keys, at most leaf_capacity + 1), its counts to counts[leaf_offsets[s] ...],
 * its nodes to node_keys / child[node_offsets[s] ...] (child indices relative
 * to the set), and its 23 level offsets to level_offsets[23 s ...].
 * results[s] receives leaf and node counts, rounds and a cstone_status (OK,
 * NONFINITE, CAPACITY, NOT_CONVERGED) for the set, or DEVICE in every set if
 * a device-side wait gave up (its arrays are then unreliable). Look-back
 * passes take their tiles in the order their blocks start, so batches (and
 * single builds) on different streams of one device may run at the same
 * time.
 */
typedef struct cstone_set {
    uint64_t n;             /* particles, 0 allowed */
    cstone_box box;
    int32_t curve;          /* cstone_curve */
    uint32_t n_crit;        /* >= 1 */
    uint64_t leaf_capacity; /* 0: cstone_leaf_capacity_bound(n, n_crit, 1) */
} cstone_set;

typedef struct cstone_set_result {
    uint32_t n_leaves, n_nodes, rounds, status;
} cstone_set_result;

typedef struct cstone_batch_layout {
    uint64_t n_sets;
    uint64_t n_particles;     /* sum of n */
    uint64_t leaf_slots;      /* entries of leaves and counts */
    uint64_t node_slots;      /* entries of node_keys and child */
    uint64_t workspace_bytes; /* for any sort shape */
    uint64_t n_tiles;         /* sort tiles of the current shape */
    int32_t sort_variant;
    uint32_t rounds;          /* rebalance rounds enqueued (rounds after convergence exit at once) */
} cstone_batch_layout;

typedef struct cstone_batch cstone_batch; /* host-side plan */

/* Plan a batch: offsets, capacities and tile tables (host memory only).
 * Errors: INVALID_ARG (n_crit 0, a bad box or curve, more than 2^32 - 1
 * particles or entries in total). */
CSTONE_API cstone_status cstone_batch_create(const cstone_set* sets, uint32_t n_sets, cstone_batch** plan);
CSTONE_API void cstone_batch_destroy(cstone_batch* plan);
/* Any of the offset arrays (host, n_sets + 1 entries) may be NULL. */
CSTONE_API cstone_status cstone_batch_get_layout(const cstone_batch* plan, cstone_batch_layout* layout,
                                      uint64_t* particle_offsets, uint64_t* leaf_offsets, uint64_t* node_offsets);
/* Sort shape of this plan (cstone_sort_variant_count() shapes; a new plan
 * takes the autotune table's shape for its size, else the built-in one); call
 * cstone_batch_upload again afterwards. */
CSTONE_API cstone_status cstone_batch_set_variant(cstone_batch* plan, int variant);
/* Rebalance rounds enqueued per build, 1 .. L + 1 = 22 (the default); a set
 * whose tree needs more reports NOT_CONVERGED. Drops a captured graph. */
CSTONE_API cstone_status cstone_batch_set_rounds(cstone_batch* plan, uint32_t rounds);
/* Copy the plan's tables into the workspace (device, layout.workspace_bytes).
 * Synchronises `stream`; needed once before building with that workspace. */
CSTONE_API cstone_status cstone_batch_upload(const cstone_batch* plan, void* ws, size_t ws_bytes, hipStream_t stream);
/* The same copy without a host synchronisation: the tables are packed into
 * `host_stage` (host memory of at least cstone_batch_table_bytes(plan) bytes,
 * page-locked so that the copy is asynchronous: hipHostMalloc) in their
 * workspace layout and copied with one asynchronous transfer on `stream`.
 * The caller keeps host_stage unchanged until the stream has passed the copy.
 * Errors: INVALID_ARG (a null pointer, a workspace or stage too small). */
CSTONE_API size_t cstone_batch_table_bytes(const cstone_batch* plan);
CSTONE_API cstone_status cstone_batch_upload_staged(const cstone_batch* plan, void* ws, size_t ws_bytes, void* host_stage,
                                                    size_t stage_bytes, hipStream_t stream);
/* Enqueue the whole batched build on `stream`; no host synchronisation, no
 * allocation, so it may be captured. Device arrays as in the layout above. */
CSTONE_API cstone_status cstone_batch_build(const cstone_batch* plan, const double* x, const double* y, const double* z,
                                 uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves, uint32_t* counts,
                                 uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                 cstone_set_result* results, void* ws, size_t ws_bytes, hipStream_t stream);
/* Capture cstone_batch_build with these arrays into a hipGraph kept by the
 * plan (replacing an earlier one). `stream` must not be the null stream. */
CSTONE_API cstone_status cstone_batch_capture(cstone_batch* plan, const double* x, const double* y, const double* z,
                                   uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves, uint32_t* counts,
                                   uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                   cstone_set_result* results, void* ws, size_t ws_bytes, hipStream_t stream);
/* Launch the captured graph on `stream` (asynchronous). */
CSTONE_API cstone_status cstone_batch_launch(cstone_batch* plan, hipStream_t stream);
/* Build with every sort shape (reps timed builds each, after one warm-up),
 * keep the fastest in the plan, upload it and record it in the autotune table
 * for (CSTONE_TUNE_BATCH_SORT, the plan's particle count, this device). Times
 * per shape (host, or NULL). Drops a captured graph. Synchronises `stream`. */
CSTONE_API cstone_status cstone_batch_autotune(cstone_batch* plan, const double* x, const double* y, const double* z,
                                    uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves, uint32_t* counts,
                                    uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                    cstone_set_result* results, void* ws, size_t ws_bytes, int reps,
                                    float* ms_per_variant, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CSTONE_H */
