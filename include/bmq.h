/*
 * bmq.h -- C ABI of the MI355X compressed state-vector stage loop.
 *
 * The library simulates a quantum circuit on a state vector that is kept
 * compressed in device memory between stages (paper: Zhang et al., "Overcoming
 * Memory Constraints in Quantum Circuit Simulation with a High-Fidelity
 * Compression Framework", arXiv 2410.14088).  The problem statement the calls
 * follow: the input is a circuit, the SV block size and the inner size
 * (Algorithm 1's "Require" line, Section 4.1) plus a codec error bound
 * (Section 5.1); the state starts at |0...0> (Section 4.2); the outputs are
 * the final state's fidelity (Section 5.3) and memory footprint (Section 5.4).
 *
 * Conventions shared by every call
 *   - Status: every int-returning call returns SV_OK (0) or a negative SV_ERR_*
 *     code; sv_last_error() gives a thread-local message.  No call throws.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary process memory.  Every call names which it takes.
 *   - Work is enqueued on the HIP stream given to sv_create (a hipStream_t
 *     passed as void*; NULL = the default stream).  Calls that return values
 *     to the host synchronise that stream before returning.
 *   - Ownership: the caller owns every buffer it passes (the device arena, the
 *     stream, input and output arrays) and keeps them alive while a handle
 *     that uses them exists.  The library owns the sv_t and sv_plan_t handles
 *     (host heap) and only sub-allocates inside the caller's arena.
 *   - Qubit q is bit q of the amplitude index (qubit 0 = least significant,
 *     Section 2.1).  With block size b the low b bits are the local index and
 *     the high c = n - b bits the global index (Section 3, Fig. 1).
 *   - Complex arrays are interleaved (re, im) pairs: complex64 = 2 x float32,
 *     complex128 = 2 x float64, amplitude i at element i.
 *   - After SV_ERR_CAPACITY or SV_ERR_CORRUPT a handle is poisoned: only
 *     sv_destroy is valid.  SV_ERR_INVALID leaves every argument untouched.
 */
#ifndef BMQ_H
#define BMQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SV_OK = 0,
    SV_ERR_INVALID = -1,      /* bad argument or configuration */
    SV_ERR_OOM = -2,          /* the caller's arena is smaller than required */
    SV_ERR_CAPACITY = -3,     /* a compressed pool overflowed during a stage */
    SV_ERR_HIP = -4,          /* a HIP runtime call failed */
    SV_ERR_CORRUPT = -5,      /* a stream or directory entry is malformed */
    SV_ERR_UNSUPPORTED = -6,  /* valid request the library does not implement */
    SV_ERR_TIMEOUT = -7       /* a bounded device-side wait ran out (persistent launch) */
};

/* Codec domains (Section 4.3).  LIN: the error bound applies to each real
 * and imaginary part directly (point-wise absolute).  LOG: Algorithm 2 --
 * sign bitmap, magnitude, log2, absolute bound eb on log2|x|, which is the
 * point-wise relative bound 2^eb - 1 of Eq. 1-2.  RAW: no compression --
 * every chunk is stored VERBATIM (raw float32, lossless; eb is not used), the
 * same stage loop without the codec, as in the no-compression comparison of
 * Section 5's compression-overhead analysis.  Only the initial state keeps
 * its all-zero chunks as ZERO directory entries. */
enum { SV_DOMAIN_LIN = 0, SV_DOMAIN_LOG = 1, SV_DOMAIN_RAW = 2 };

/* Gate kinds.  1-qubit matrices as usual; for 2-qubit gates the 4x4 matrix
 * index is 2*bit(q[0]) + bit(q[1]), the row order of Section 2.1.
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]]
 *   RX(b) = [[c, -i s], [-i s, c]], RY(t) = [[c, -s], [s, c]],
 *   RZ(t) = diag(e^{-it/2}, e^{it/2}), CX: control q[0], target q[1],
 *   CZ = diag(1,1,1,-1), CP(l) = diag(1,1,1,e^{il}),
 *   RZZ(g) = diag(e^{-ig/2}, e^{ig/2}, e^{ig/2}, e^{-ig/2}). */
enum {
    SV_GATE_H = 0, SV_GATE_X, SV_GATE_Y, SV_GATE_Z, SV_GATE_S, SV_GATE_T,
    SV_GATE_RX, SV_GATE_RY, SV_GATE_RZ, SV_GATE_U3,
    SV_GATE_CX, SV_GATE_CZ, SV_GATE_CP, SV_GATE_RZZ, SV_GATE_COUNT
};

typedef struct {
    int32_t kind;      /* SV_GATE_* */
    int32_t q[2];      /* qubits; q[1] unused for 1-qubit gates */
    int32_t pad;
    double p[3];       /* angles in radians (U3: theta, phi, lambda) */
} sv_gate_t;

typedef struct {
    int32_t n_qubits;     /* n, 10..40 */
    int32_t block_qubits; /* b: SV block = 2^b amplitudes, 6 <= b <= n */
    int32_t inner_size;   /* Algorithm 1 inner size; threshold = max(inner, 2) */
    int32_t fuse_qubits;  /* widest dense fused gate, 1..5 */
    int32_t domain;       /* SV_DOMAIN_LIN, SV_DOMAIN_LOG or SV_DOMAIN_RAW */
    int32_t tile_qubits;  /* amplitudes per on-chip tile = 2^tile_qubits; 0 = default (12) */
    double eb;            /* absolute bound in the codec domain, > 0 */
    uint64_t pool_bytes;  /* device capacity of each compressed pool; 0 = worst case */
    uint32_t flags;       /* SV_FLAG_* */
    uint32_t reserved;    /* 0 */
} sv_config_t;

/* SV_FLAG_NO_SCRATCH: no uncompressed scratch planes in the arena (they are
 * as large as the uncompressed state).  A stage that needs several tile
 * passes then recompresses between passes, i.e. runs as several compressed
 * sub-stages: less device memory, one more compression per extra pass. */
#define SV_FLAG_NO_SCRATCH 1u
/* SV_FLAG_NO_MFMA: apply dense 4- and 5-qubit fused operations with vector
 * FMAs instead of the matrix cores (for comparison; both are float32). */
#define SV_FLAG_NO_MFMA 2u
/* SV_FLAG_GATE_PER_STAGE: planning only (a state accepts plans with or
 * without it).  Every gate becomes a stage of its own, so the whole state is
 * decompressed, updated by one gate and recompressed once per gate: the basic
 * per-gate workflow that Section 3 contrasts with Algorithm 1, kept for the
 * ablation of compression count against fidelity and time. */
#define SV_FLAG_GATE_PER_STAGE 4u
/* SV_FLAG_DIAGONAL_FREE: planning only.  Algorithm 1 counts only the global
 * indices of non-diagonal gates.  A diagonal gate (Z, S, T, RZ, CZ, CP, RZZ)
 * multiplies each amplitude by a phase fixed by that amplitude's own index
 * bits, so it never pairs two SV blocks (the two-block case of Section 3's
 * update rules does not arise) and runs inside any group: fewer stages, so
 * fewer compressions.  The planner variant that Section 4.1's goal (as few
 * compressions as possible) suggests; ignored with SV_FLAG_GATE_PER_STAGE. */
#define SV_FLAG_DIAGONAL_FREE 8u
/* SV_FLAG_COMMUTE: planning only.  Algorithm 1 with commutation: a stage
 * takes, in input order, every remaining gate that fits the threshold and
 * commutes with each remaining gate it overtakes (disjoint qubits, or both
 * diagonal: the reordered circuit has the same unitary); the gates it defers
 * form the next stage's candidates.  Fewer stages, so fewer compressions
 * (Section 4.1's goal).  The plan's gate order then differs from the input
 * order: plan_stage ranges index the plan order, plan_gate_order maps it
 * back.  Combines with SV_FLAG_DIAGONAL_FREE; ignored with
 * SV_FLAG_GATE_PER_STAGE. */
#define SV_FLAG_COMMUTE 16u
/* SV_FLAG_GROUP_SCRATCH: the scratch planes hold one SV group instead of the
 * whole state.  A stage that needs several tile passes then runs all of its
 * passes group by group (Section 4.2: the groups of a stage are independent),
 * so the planes shrink from 2^n to 2^max(b + max(inner, 2), tile) amplitudes
 * each (e.g. 512 MiB instead of 64 GiB per plane pair at n = 33, b = 24).
 * Same records as full scratch planes.  A plan whose multi-pass stage spans
 * more qubits than that (a larger inner size or tile) is refused with
 * SV_ERR_INVALID; batched and whole-circuit queue launches refuse such
 * states when a stage has several passes (SV_ERR_UNSUPPORTED).  Ignored with
 * SV_FLAG_NO_SCRATCH. */
#define SV_FLAG_GROUP_SCRATCH 32u
/* SV_FLAG_REMAP: planning only.  Algorithm 1 with qubit remapping (Section
 * 4.1's goal of fewer stages, so fewer compressions): logical qubits move
 * between bit positions of the amplitude index.  Where the next gate would
 * exceed the threshold, before the stage is closed, each inner (global)
 * position of the stage, ascending, whose logical qubit is used again is
 * swapped with the local position whose logical qubit is next used last
 * (ties: the lowest position), if that use comes strictly later; the swap is
 * appended to the stage as CX(l, g) CX(g, l) CX(l, g) (both positions are
 * already in the stage).  Later gates act on their qubits' new positions.
 * The plan's gates are then the physical circuit (plan_gate; plan_gate_order
 * gives 0xFFFFFFFF for the swap gates) and the state ends with logical qubit
 * L at position plan_layout[L]: amplitude x of the circuit's state is
 * amplitude pi(x) of the simulated state, pi moving bit L to bit
 * plan_layout[L] (pi(0) = 0).  Combines with SV_FLAG_DIAGONAL_FREE, not with
 * SV_FLAG_GATE_PER_STAGE or SV_FLAG_COMMUTE (SV_ERR_INVALID). */
#define SV_FLAG_REMAP 64u

/* Per-stage statistics (all counts over the whole state). */
typedef struct {
    uint64_t bytes_in;        /* compressed record bytes the stage read (first pass) */
    uint64_t bytes_out;       /* compressed record bytes the stage wrote (last pass) */
    uint64_t bytes_out_host;  /* of bytes_out, those placed in the host pool */
    uint64_t inter_bytes;     /* compressed bytes written and read back between passes */
    uint64_t dir_bytes;       /* directory bytes read + written */
    uint64_t scratch_bytes;   /* uncompressed scratch bytes read + written */
    uint64_t zero_chunks_out; /* 64-amplitude chunks that are entirely zero */
    uint64_t mode_hist[4];    /* plane-chunks per mode: ZERO, LZ, Q0, VERBATIM */
    uint32_t passes;          /* on-chip tile passes of the stage */
    uint32_t n_ops;           /* fused operations applied */
    uint32_t n_gates;         /* circuit gates in the stage */
    uint32_t n_inner;         /* inner (global) indices of the stage */
    float ms;                 /* device time of the stage's kernels (HIP events) */
    uint32_t launches;        /* pass-kernel launches: passes, or passes x groups with group-sized scratch */
} sv_stage_stats_t;

typedef struct sv_plan sv_plan_t;
typedef struct sv_state sv_t;
typedef struct sv_graph sv_graph_t;

/* Thread-local text of the last error (never NULL). */
const char *sv_last_error(void);

/* ---------------------------------------------------------------- planning
 * stage_plan -- Algorithm 1 (Section 4.1): cut the gate list, in order, into
 * stages whose gates touch at most max(inner_size, 2) global indices; the
 * global indices a stage touches are its inner indices, the rest are outer,
 * and the blocks sharing the outer bits form an SV group (2^(c-m) groups of
 * 2^m blocks for m inner indices).  Then, per stage, lay out the on-chip tile
 * passes and fuse consecutive gates into dense (<= fuse_qubits) and diagonal
 * operations.  Host only, deterministic.
 *   gates: host array of n_gates gates, copied.  cfg: host, copied.
 *   out:   receives a new plan; free with plan_destroy.
 * Errors: SV_ERR_INVALID for a bad config, a bad gate or a gate that touches
 * more global indices than the threshold. */
int stage_plan(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg,
               sv_plan_t **out);

/* Plan summary: stages, fused operations and tile passes (any may be NULL). */
int plan_info(const sv_plan_t *p, size_t *n_stages, size_t *n_ops, size_t *n_passes);

/* Stage s: its gate range [gate_begin, gate_end) in the plan's gate order,
 * its inner indices (up to 8 written to inner_out, count in n_inner) and its
 * number of tile passes. */
/* plan_layout -- phys_of_logical[L] (host, n = n_qubits entries) receives the
 * bit position of logical qubit L after the plan (identity unless
 * SV_FLAG_REMAP).  plan_gate -- the plan's k-th gate as applied (kind, the
 * bit positions it acts on -- qubits[1] = -1 for one-qubit gates -- and its
 * three parameters); any output may be NULL. */
int plan_layout(const sv_plan_t *p, int32_t *phys_of_logical, size_t n);
int plan_gate(const sv_plan_t *p, size_t k, int32_t *kind, int32_t *qubits, double *params);

int plan_stage(const sv_plan_t *p, size_t s, size_t *gate_begin, size_t *gate_end,
               int32_t *inner_out, int32_t *n_inner, int32_t *n_passes);

/* plan_gate_order -- order_out[k] (host, n = the plan's gate count, i.e. the
 * last stage's gate_end) receives the input index of the plan's k-th gate:
 * the identity unless the plan was made with SV_FLAG_COMMUTE or
 * SV_FLAG_REMAP (0xFFFFFFFF for a remapping swap gate). */
int plan_gate_order(const sv_plan_t *p, uint32_t *order_out, size_t n);

/* plan_stage_ops -- the fused operations of stage s are plan operations
 * [op_begin, op_end), applied in that order (pass after pass).
 * plan_op -- read-only view of plan operation i, for checking the fusion on
 * the host: type (0 dense, 1 diagonal), k qubits written to qubits[0..k)
 * (operation qubit j is bit j of the matrix or table index), and, when
 * data_host is not NULL, its complex64 values (interleaved float32 pairs):
 * dense, the 2^k x 2^k matrix row major; diagonal, the 2^k phases.
 * cap_elems is data_host's capacity in complex64 values (SV_ERR_INVALID when
 * too small). */
int plan_stage_ops(const sv_plan_t *p, size_t s, size_t *op_begin, size_t *op_end);
int plan_op(const sv_plan_t *p, size_t i, int32_t *type, int32_t *k, int32_t *qubits, void *data_host,
            size_t cap_elems);

void plan_destroy(sv_plan_t *p);

/* ---------------------------------------------------------------- state
 * sv_mem_required -- bytes of device arena sv_create needs for cfg:
 * two chunk directories and two compressed record pools of pool_bytes each
 * (the stage loop reads one and writes the other), the uncompressed scratch
 * planes for multi-pass stages (none with SV_FLAG_NO_SCRATCH), the operation
 * arena and reduction buffers. */
int sv_mem_required(const sv_config_t *cfg, uint64_t *bytes);

/* sv_create -- bind the caller's device arena (dev_arena, dev_bytes; 256-byte
 * aligned) and stream, and set the state to |0...0> (Section 4.2): the first
 * 64-amplitude chunk (amplitude 0 = 1) is encoded on the device and every
 * other chunk's directory entry points at the shared all-zero record, the
 * directory analogue of compressing one zero block and copying it.
 * Errors: SV_ERR_INVALID (config), SV_ERR_OOM (arena too small), SV_ERR_HIP. */
int sv_create(const sv_config_t *cfg, void *dev_arena, uint64_t dev_bytes,
              void *hip_stream, sv_t **out);

void sv_destroy(sv_t *sv);

/* sv_attach_host_pool -- the second memory level (Section 4.4 two-level
 * memory management): host_pinned is page-locked host memory the device can
 * address (hipHostMalloc, or a pinned torch tensor), of host_bytes; it is
 * split into two halves that pair with the two device pools.  When a device
 * pool segment is full, a wave's record bodies go to the host half instead;
 * directory offsets at and above pool_bytes address the host half.  Kernels
 * read and write it in place over the host link.  The caller owns the memory
 * and keeps it alive while the state exists.  Passing NULL, 0 detaches it.
 * Errors: SV_ERR_INVALID (not device-addressable, too small, or the live
 * state still has records in the attached host pool). */
int sv_attach_host_pool(sv_t *sv, void *host_pinned, uint64_t host_bytes);

/* sv_host_alloc -- page-locked, device-addressable host memory of exactly
 * `bytes` (hipHostMalloc), for sv_attach_host_pool and the pipeline's host
 * store: a host pool sized to a memory budget must not be rounded up (a
 * caching pinned allocator that rounds to a power of two nearly doubles a
 * 150 GB request).  *ptr receives the host address; the caller frees it
 * with sv_host_free once no state uses it.  Errors: SV_ERR_INVALID (bytes
 * is 0 or ptr NULL), SV_ERR_HIP (the allocation failed; *ptr is NULL).
 * sv_host_free(NULL) does nothing. */
int sv_host_alloc(uint64_t bytes, void **ptr);
int sv_host_free(void *ptr);

/* sv_reset -- set an existing state back to |0...0> (as sv_create does),
 * enqueued on its stream without synchronising. */
int sv_reset(sv_t *sv);

/* stage_apply_compressed -- the per-stage block loop: for stages
 * [first, first+count) of plan p, every tile of every SV group is decoded from
 * the compressed pool into on-chip memory, every fused operation of the stage
 * is applied, and the tile is re-encoded by the point-wise error-bounded codec
 * into the other pool (Sections 4.1-4.3).  One compression per stage.
 * stats: NULL, or host array of count entries; when given, each stage's
 * kernels are bracketed by HIP events and the call synchronises.
 * The plan must have been made with a config whose n, b, domain and eb equal
 * the state's.  Errors: SV_ERR_INVALID, SV_ERR_CAPACITY (the device pool and
 * the host pool, if any, overflowed: raise pool_bytes or attach a larger host
 * pool), SV_ERR_HIP. */
int stage_apply_compressed(sv_t *sv, const sv_plan_t *p, size_t first, size_t count,
                           sv_stage_stats_t *stats);

/* sv_autotune -- choose tile_qubits (10..13, <= n) and fuse_qubits (1..5)
 * for a circuit by measurement: each candidate is planned, run from |0...0>
 * for its first probe_stages stages (all if 0) on the caller's arena and
 * stream (once to warm up, once timed with HIP events), and the fastest wins.
 * Candidates that overflow the pools are skipped.  The arena must hold
 * sv_mem_required(cfg) bytes (the same for every candidate); its contents are
 * overwritten.  best: receives cfg with the winning tile_qubits and
 * fuse_qubits.  ms_all: NULL or 20 floats, entry (tile-10)*5 + (fuse-1) = the
 * candidate's time in ms, NaN when not run.  Synchronises. */
int sv_autotune(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg, void *dev_arena,
                uint64_t dev_bytes, void *hip_stream, size_t probe_stages, sv_config_t *best,
                float *ms_all);

/* sv_autotune_space -- the same measurement over a caller-chosen search
 * space: every combination of the tile sizes, fusion widths and inner sizes
 * (Algorithm 1's inner size, which sets how many global indices a stage may
 * hold and so the number of stages; the parameter study of Section 5 varies
 * it with the block size).  Each candidate is planned on the first
 * probe_gates gates of the circuit (all if 0), run once to warm up and once
 * timed from |0...0>; candidates whose plan is invalid (a gate wider than
 * the inner size allows) or whose records overflow the pools are skipped.
 * The arena must hold sv_mem_required(cfg) bytes (tile, fusion width and
 * inner size do not change it); its contents are overwritten.  best: cfg
 * with the winning tile_qubits, fuse_qubits and inner_size.  ms_out: NULL or
 * n_tiles * n_fuse * n_inner floats, entry (it * n_fuse + ifu) * n_inner + ii
 * = the time of (tiles[it], fuse[ifu], inner[ii]) in ms, NaN when not run.
 * sv_autotune is this function over tiles 10..min(13, n), fusion widths 1..5
 * and the configuration's inner size.  Synchronises. */
typedef struct {
    int32_t n_tiles, tiles[4];      /* tile_qubits candidates, 10..13 */
    int32_t n_fuse, fuse[5];        /* fuse_qubits candidates, 1..5 */
    int32_t n_inner, inner[6];      /* inner_size candidates, 1..8 */
    uint64_t probe_gates;           /* prefix of the circuit that is timed (0: all of it) */
} sv_tune_space_t;
int sv_autotune_space(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg, void *dev_arena,
                      uint64_t dev_bytes, void *hip_stream, const sv_tune_space_t *space, sv_config_t *best,
                      float *ms_out);

/* ---------------------------------------------------------------- graphs
 * sv_graph_capture -- record the stage loop of stages [first, first+count)
 * of plan p on state sv (counter clearing plus every tile pass, as
 * stage_apply_compressed would enqueue them) into a HIP graph, without running
 * it.  At most 512 pass launches.  The graph is tied to sv, to p's uploaded
 * operations and to the state's current pool copy: it may be replayed when
 * the state is in that copy again (after sv_reset, or after an even number
 * of compressed passes).  Not available while a debug dump is set.
 * sv_graph_launch -- replay on the state's stream, asynchronously.  The
 * replay's overflow check and footprint update happen at the next
 * sv_graph_sync, stage_apply_compressed, sv_footprint or another replay.
 * sv_graph_sync -- synchronise and run that check (SV_ERR_CAPACITY on
 * overflow).  sv_graph_destroy -- free the graph (p and sv must still exist). */
int sv_graph_capture(sv_t *sv, const sv_plan_t *p, size_t first, size_t count, sv_graph_t **out);
int sv_graph_launch(sv_t *sv, sv_graph_t *g);
int sv_graph_sync(sv_t *sv);
void sv_graph_destroy(sv_graph_t *g);

/* ---------------------------------------------------------------- host-resident pipeline
 * The paper's deployment (Section 4.2, Fig. 6): the compressed state lives in
 * pinned host memory and every stage moves each SV group through the GPU --
 * copy its blocks in, decompress / apply / recompress, copy them back -- with
 * the groups spread over S streams so that one group's copies overlap
 * another's kernels (the stream-count study of Section 5 varies S).
 *
 * Host store: one image per SV block, [the block's 2^(b-6) directory entries,
 * body offsets relative to the image's body area] [record bodies in chunk
 * order] (the record format of the codec), in the caller's pinned buffer.  A
 * block's new image overwrites its old one when it fits, else it takes a new
 * slot with a quarter of headroom (bump allocation; sv_pipe_reset starts
 * over), so the store stays near the live compressed bytes.  Device: per
 * stream, staging for one group (input and output directories and pools,
 * group-sized scratch planes, packing buffers) plus the plan's operations.
 * Records are bit-identical to stage_apply_compressed on a device state.
 *
 * sv_pipe_required -- device workspace bytes for cfg and `streams` (1..8),
 *   and the smallest host store (the initial state; a run needs about
 *   1.25 x the largest compressed state plus 8 bytes per 64 amplitudes).
 * sv_pipe_create -- bind the device workspace (256-byte aligned, caller-owned)
 *   and the pinned host store (hipHostMalloc or torch pin_memory, 256-byte
 *   aligned; the library never registers or frees it), create the streams
 *   (default priority), and set |0...0>.  SV_DOMAIN_RAW is refused.  Groups
 *   span block_qubits + max(inner_size, 2) qubits (at least a tile).
 * sv_pipe_reset -- back to |0...0>; the host store is reused from its start.
 * sv_pipe_apply -- stages [first, first + count) of p; waits for earlier work
 *   on hip_stream first and returns when every image is back in the host
 *   store.  stats (nullable, count entries): ms = wall time of the stage,
 *   bytes_in / bytes_out = bytes copied in / out, passes, gates, ops.
 *   SV_ERR_CAPACITY (poisoned) when the host store is full; SV_ERR_INVALID
 *   when a stage spans more qubits than the staging holds; SV_ERR_UNSUPPORTED
 *   for multi-pass stages with SV_FLAG_NO_SCRATCH.
 * sv_pipe_load -- copy the host-resident state into a device state of the same
 *   n, b, domain and eb (its directory and current pool copy), e.g. to read or
 *   check it with sv_fidelity / sv_block_stream.  Synchronises.
 * sv_pipe_footprint -- record bytes, image bytes (records + directories),
 *   host store bytes in use, and bytes copied in / out since the last reset.
 * sv_pipe_destroy -- synchronise, destroy the streams, free the handle. */
typedef struct sv_pipe sv_pipe_t;
int sv_pipe_required(const sv_config_t *cfg, int32_t streams, uint64_t *dev_bytes, uint64_t *host_min_bytes);
int sv_pipe_create(const sv_config_t *cfg, int32_t streams, void *dev_ws, uint64_t dev_bytes, void *host_pinned,
                   uint64_t host_bytes, void *hip_stream, sv_pipe_t **out);
int sv_pipe_reset(sv_pipe_t *pp);
int sv_pipe_apply(sv_pipe_t *pp, const sv_plan_t *p, size_t first, size_t count, sv_stage_stats_t *stats);
int sv_pipe_load(sv_pipe_t *pp, sv_t *sv);
int sv_pipe_footprint(const sv_pipe_t *pp, uint64_t *record_bytes, uint64_t *image_bytes, uint64_t *host_used,
                      uint64_t *h2d_bytes, uint64_t *d2h_bytes);
void sv_pipe_destroy(sv_pipe_t *pp);

/* ---------------------------------------------------------------- batches
 * sv_batch_apply -- run every stage of plans[i] on states[i] for count
 * independent circuits together: launch k executes the k-th tile pass of
 * every circuit that has one, in one grid over all their tiles (one grid per
 * tile size), so small circuits share the device instead of running one
 * after another.  Each state ends exactly as stage_apply_compressed would
 * leave it (same kernels, same records).  All states must use hip_stream;
 * each circuit may need at most 512 pass launches.  workspace_dev: device
 * memory, 256-byte aligned, of sv_batch_workspace bytes (launch arguments).
 * Synchronises; on overflow the overflowing states are poisoned and the
 * first error is returned. */
int sv_batch_workspace(sv_t *const *states, const sv_plan_t *const *plans, size_t count,
                       uint64_t *bytes);
int sv_batch_apply(sv_t *const *states, const sv_plan_t *const *plans, size_t count,
                   void *workspace_dev, uint64_t workspace_bytes, void *hip_stream);

/* sv_persistent_apply -- the work of sv_batch_apply (every stage of
 * plans[i] on states[i]) in ONE launch per tile size and codec domain
 * instead of one launch per pass step.  Stages run one after another because
 * each reads every block the previous one wrote (Section 4.2 workflow, Fig. 6);
 * here the stage boundary is a per-circuit barrier inside the launch:
 * workgroups take items (runs of consecutive tiles of one pass) from a
 * device queue in pass order, and an item of pass k of a circuit starts once
 * every item of that circuit's pass k - 1 is done (atomic counters), so
 * circuits advance independently and a workgroup never waits for the launch
 * to end.  Results are identical to
 * sv_batch_apply and stage_apply_compressed (same pass body, same records).
 * wait_limit_us bounds every device-side wait (0 = 10 s): a wait that runs
 * out aborts the whole launch, which always finishes; the states of an
 * aborted launch are poisoned (sv_reset clears that) and SV_ERR_TIMEOUT is
 * returned.  Same arguments, checks, limits and ownership as sv_batch_apply;
 * workspace_dev: device memory, 256-byte aligned, of sv_persistent_workspace
 * bytes (launch arguments, queue and counters).  Synchronises. */
int sv_persistent_workspace(sv_t *const *states, const sv_plan_t *const *plans, size_t count,
                            uint64_t *bytes);
/* sv_graph_capture_persistent -- the whole-circuit queue launch of every
 * stage of plan p on state sv, recorded into a HIP graph without running it:
 * the preparation (plan upload and the workspace image: launch arguments,
 * queue tables) happens now, once, and the graph holds only kernels (the
 * counter and queue-word clears as fill kernels, then the queue kernel), so
 * that one replay runs the whole circuit.  workspace_dev: as for
 * sv_persistent_apply (sv_persistent_workspace bytes for {sv}, {p}); it must
 * stay alive and unchanged while the graph exists.  Replay with
 * sv_graph_launch (the state must be in the pool copy it was captured in:
 * after sv_reset, or an even number of compressed passes later); the abort
 * flags and the stage counters are read at the next synchronising call
 * (SV_ERR_TIMEOUT, state poisoned, when a bounded wait ran out). */
int sv_graph_capture_persistent(sv_t *sv, const sv_plan_t *p, void *workspace_dev, uint64_t workspace_bytes,
                                uint32_t wait_limit_us, sv_graph_t **out);
int sv_persistent_apply(sv_t *const *states, const sv_plan_t *const *plans, size_t count,
                        void *workspace_dev, uint64_t workspace_bytes, uint32_t wait_limit_us,
                        void *hip_stream);

/* sv_fidelity -- FP64 reductions on the device (Section 5.3 fidelity; the
 * paper prints the unsquared |<ref|psi>|).  The reference is one of:
 *   ref_host: host array of 2^n complex128 (interleaved), streamed to the
 *             device slice by slice through the state's staging area;
 *   ref_dev:  device array of 2^n complex128;
 *   ref_sv:   a second compressed state of the same n (any domain), decoded
 *             beside sv;
 *   none:     only norm2 is computed (the other fields are NaN).
 * out receives
 *   overlap2    = |<ref|psi>|^2 with reference and state as they are: the
 *                 squared fidelity, which also counts any norm the codec
 *                 loses or gains;
 *   fidelity    = |<ref|psi>|^2 / (|ref|^2 |psi|^2), both sides normalised;
 *   overlap_re, overlap_im = <ref|psi>;
 *   max_abs_err = max over amplitudes and over re/im of |psi - ref|;
 *   norm2 = |psi|^2, ref_norm2 = |ref|^2.
 * Errors: SV_ERR_INVALID (more than one reference, n differs).  Synchronises
 * (and, for ref_sv on another stream, synchronises that stream first). */
typedef struct {
    double overlap2, fidelity, overlap_re, overlap_im, max_abs_err, norm2, ref_norm2;
} sv_fidelity_t;
int sv_fidelity(const sv_t *sv, const double *ref_host, const double *ref_dev, const sv_t *ref_sv,
                sv_fidelity_t *out);

/* sv_sample -- draw k amplitude indices x with probability |psi(x)|^2 /
 * |psi|^2 (the measurement distribution; feeds the importance-sampled
 * fidelity estimate <psi|ref> = |psi|^2 E_x[ref(x) / psi(x)] when the
 * reference is known only amplitude by amplitude).  Two levels on the
 * device: |psi|^2 per group of 2^max(10, n-16) amplitudes, then, per
 * sample, a walk through the chosen group in index order with a running
 * FP64 sum.  The uniforms are u_i = output i (i = 0, 1, ...) of SplitMix64
 * started at `seed` (Steele, Lea and Flood, OOPSLA 2014), top 53 bits.
 * idx_host: host array of k indices.  Errors: SV_ERR_INVALID (NULL output,
 * a state of zero or non-finite norm).  Synchronises. */
int sv_sample(const sv_t *sv, uint64_t k, uint64_t seed, uint64_t *idx_host);

/* sv_export -- decode amplitudes [start, start+count) into dst_dev
 * (device, count complex64).  start and count must be multiples of 64. */
int sv_export(const sv_t *sv, uint64_t start, uint64_t count, void *dst_dev);

/* sv_amplitudes -- decode the k amplitudes at idx_dev[0..k) (device uint64)
 * into out_dev (device, k complex64). */
int sv_amplitudes(const sv_t *sv, const uint64_t *idx_dev, uint64_t k, void *out_dev);

/* sv_footprint -- current compressed footprint (Section 5.4 memory metric):
 * record bytes of the live state copy (device and host pools together), of
 * those the bytes in the host pool, and directory bytes.  Synchronises.
 * Any output pointer may be NULL. */
int sv_footprint(const sv_t *sv, uint64_t *record_bytes, uint64_t *host_bytes, uint64_t *dir_bytes);

/* sv_check -- validate the live state copy's chunk directory on the device
 * (the stage loop itself trusts it and does not): every entry must be 0 (an
 * all-zero chunk) or carry two well-formed plane headers for the state's
 * codec domain (the record format of Section 4.3's codec: mode, width <= 32,
 * sign class not 3, zero class 0 or 2, no sign or zero class in LIN, no
 * packed plane in RAW) and the offset of a record that lies inside the pool
 * it names (device pool, or the attached host pool's half).  *n_bad (may be
 * NULL) receives the number of bad entries.  Returns SV_OK, or
 * SV_ERR_CORRUPT with the state poisoned.  Synchronises.
 * sv_directory -- a read-only diagnostic view of that directory: its device
 * address (*dir_dev, one u64 per 64-amplitude chunk: body offset in bits
 * 39:0, real-plane header in 51:40, imaginary-plane header in 63:52) and its
 * number of entries.  Valid until the next call that runs a stage. */
int sv_check(sv_t *sv, uint64_t *n_bad);
int sv_directory(const sv_t *sv, const uint64_t **dir_dev, uint64_t *n_entries);

/* sv_block_stream -- the canonical stream of SV block `block` (2^b
 * amplitudes): a 16-byte block header (u8 0x51, u8 version 1, u8 domain,
 * u8 log2 chunk = 6, u32 eb float bits, u32 n_values, u32 n_chunks) followed
 * by the records of its chunks in index order (an all-zero chunk is the
 * 8-byte record of two zero headers).  dst_host: host buffer of cap bytes;
 * *bytes receives the stream size (also when cap is too small, which returns
 * SV_ERR_INVALID).  For bit-exact comparison with a reference codec. */
int sv_block_stream(const sv_t *sv, uint64_t block, void *dst_host, uint64_t cap,
                    uint64_t *bytes);

/* sv_debug_dump -- test hook: every later stage also stores, for the
 * amplitudes [start, start+count) (64-aligned), the values it is about to
 * encode (after its last fused operation, before quantization) into
 * pre_re/pre_im, and the values its first pass decoded (before any fused
 * operation) into post_re/post_im: device float32 arrays of count entries,
 * element i = amplitude start + i.  Either pair may be NULL; NULL for both
 * turns the hook off.  Not available in batched, persistent or captured
 * launches (SV_ERR_UNSUPPORTED there). */
int sv_debug_dump(sv_t *sv, uint64_t start, uint64_t count, float *pre_re, float *pre_im, float *post_re,
                  float *post_im);

/* ---------------------------------------------------------------- codec
 * The stage loop's codec (Section 4.3, Algorithm 2; the same device encoder
 * and decoder the stage loop runs) on caller arrays of whole 64-value
 * chunks: n_values must be a multiple of 64, at most 2^31.  Uses
 * cfg->domain and cfg->eb only.
 *
 * codec_encode -- the canonical block stream of the planes re_dev, im_dev
 * (device float32, n_values each): a 16-byte header (u8 0x51, u8 version
 * 1, u8 domain, u8 log2 chunk = 6, u32 eb float bits, u32 n_values, u32
 * n_chunks) followed by every chunk's record (two 32-bit plane headers,
 * then the body) in chunk order -- the stream sv_block_stream returns for an
 * SV block.  dst_dev: device, 4-byte aligned, cap bytes; *bytes receives the
 * stream size.  work_dev: device scratch of codec_workspace(n_values) bytes,
 * 256-byte aligned (record sizes and offsets).  Errors: SV_ERR_INVALID
 * (arguments; or the stream is larger than cap: *bytes is still set and
 * nothing is written).  Synchronises.
 * codec_decode -- the inverse: n_values of each plane from a stream of
 * `bytes` bytes (device, 4-byte aligned; the decoder reads packed fields as
 * 8-byte words, so up to 4 bytes past the stream's end must be readable:
 * allocate at least bytes + 4).  A one-lane walk over the record
 * headers finds the records, then they are decoded in parallel.  Errors:
 * SV_ERR_CORRUPT (header does not match cfg / n_values, a malformed plane
 * header, a record outside the stream or bytes left over).  Synchronises
 * once (the walk's verdict); the decode itself is enqueued. */
int codec_workspace(uint64_t n_values, uint64_t *bytes);
int codec_encode(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg, void *dst_dev,
                 uint64_t cap, uint64_t *bytes, void *work_dev, uint64_t work_bytes, void *hip_stream);
int codec_decode(const void *src_dev, uint64_t bytes, const sv_config_t *cfg, uint64_t n_values, float *re_dev,
                 float *im_dev, void *work_dev, uint64_t work_bytes, void *hip_stream);

/* codec_encode_noalloc -- codec_encode for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc): the
 * same stream, with the workspace in a static device array of the library
 * (4 MiB, held by every GPU the library runs on until the process ends)
 * instead of work_dev.  At most 2^24 values (SV_NOALLOC_MAX_VALUES); larger
 * inputs return SV_ERR_INVALID.  Allocates nothing (no hipMalloc, hipFree
 * or allocating library call).  Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents (nothing in it needs to start
 * at zero): calls that overlap on one GPU, on any streams, race.  Otherwise
 * as codec_encode (synchronises hip_stream). */
#define SV_NOALLOC_MAX_VALUES (1ull << 24)
int codec_encode_noalloc(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg,
                         void *dst_dev, uint64_t cap, uint64_t *bytes, void *hip_stream);

/* Slot form, for per-chunk checks: chunk i's record is written to
 * slots_dev + i*SV_CHUNK_SLOT_BYTES (device) and its size to sizes_dev[i]
 * (device uint32).  Enqueued on hip_stream; does not synchronise.
 * Errors: SV_ERR_INVALID (n_values not a multiple of 64, NULL pointers). */
#define SV_CHUNK_SLOT_BYTES 576
int codec_encode_chunks(const float *re_dev, const float *im_dev, uint64_t n_values,
                        const sv_config_t *cfg, void *slots_dev, uint32_t *sizes_dev,
                        void *hip_stream);

/* Inverse of codec_encode_chunks: decode every slot into re_dev / im_dev. */
int codec_decode_chunks(const void *slots_dev, uint64_t n_values, const sv_config_t *cfg,
                        float *re_dev, float *im_dev, void *hip_stream);

/* ---------------------------------------------------------------- predictor
 * The compression ratio of a block is unknown until it is compressed, which
 * makes device memory hard to plan (Section 3 feasibility analysis, Section
 * 4.4 two-level memory management).  A small multilayer perceptron predicts,
 * per SV block and before a stage runs, log2 of the block's stream bytes
 * after the stage and its most frequent codec mode, from features of the
 * block's current compressed form and of the stage.  It is trained online
 * with Adam on the labels each stage produces.
 *
 * Features (SV_FEATURES floats per block, from the directory headers only):
 *   0 log2 stream bytes; 1-4 fraction of planes in mode ZERO, LZ, Q0,
 *   VERBATIM; 5-12 / 13-20 width histogram (bins of 4 bits, last bin 28-32)
 *   of packed real / imaginary planes; 21 all-zero chunk fraction; 22
 *   mixed-sign fraction of packed planes; 23 / 24 mean width / 32 of packed
 *   real / imaginary planes; 25 non-diagonal gates / 64; 26 diagonal gates /
 *   64; 27 gates touching a global qubit / 64; 28 distinct local qubits
 *   touched / b; 29 fused operations / 16; 30 stage index / stages;
 *   31 log2(eb) / 32.
 * A block's stream bytes are those of sv_block_stream without its 16-byte
 * header (two 4-byte headers per chunk plus the record bodies). */
#define SV_FEATURES 32
#define SV_MLP_IN 32
#define SV_MLP_HIDDEN 64
#define SV_MLP_OUT 5
/* parameters, float32: W1[64][32] b1[64] W2[64][64] b2[64] W3[5][64] b3[5]
 * (row = output unit); ReLU after layers 1 and 2; output 0 also adds input 0
 * (the block's current log2 bytes), so the untrained net predicts no change */
#define SV_MLP_NPARAM 6597
#define SV_MLP_BETA1 0.9f
#define SV_MLP_BETA2 0.999f
#define SV_MLP_EPS 1e-8f

/* sv_block_features -- features of every block of the current state for the
 * upcoming stage `stage` of plan p.  feats_dev: device float32 array of
 * 2^(n-b) x SV_FEATURES.  Enqueued on the state's stream. */
int sv_block_features(const sv_t *sv, const sv_plan_t *p, size_t stage, float *feats_dev);

/* sv_block_labels -- per block of the current state: log2 of its stream
 * bytes (log2_bytes_dev, float32) and its most frequent plane mode
 * (mode_dev, int32 0..3; ties go to the lower mode).  Device arrays of
 * 2^(n-b) entries.  Enqueued on the state's stream. */
int sv_block_labels(const sv_t *sv, float *log2_bytes_dev, int32_t *mode_dev);

/* mlp_forward -- out_dev[batch][5] = MLP(x_dev[batch][32]).  Device arrays;
 * batch <= 2^30. */
int mlp_forward(const float *params_dev, const float *x_dev, uint32_t batch, float *out_dev,
                void *hip_stream);

/* mlp_work_floats -- floats of work space mlp_loss_grad needs for a batch. */
uint64_t mlp_work_floats(uint32_t batch);

/* mlp_loss_grad -- mean loss over the batch, 0.5 (out0 - y)^2 + cross
 * entropy of out1..4 against mode (clamped to 0..3), into loss_dev[0], and
 * its gradient with respect to the parameters into grad_dev[SV_MLP_NPARAM].
 * work_dev: mlp_work_floats(batch) floats.  1 <= batch <= 2^30.  Sums over
 * the batch run in sample order (reproducible). */
int mlp_loss_grad(const float *params_dev, const float *x_dev, const float *y_log2_bytes_dev,
                  const int32_t *y_mode_dev, uint32_t batch, float *work_dev, float *grad_dev,
                  float *loss_dev, void *hip_stream);

/* mlp_adam_update -- one Adam step (beta1 SV_MLP_BETA1, beta2 SV_MLP_BETA2,
 * eps SV_MLP_EPS, bias-corrected with step t >= 1) of params_dev with
 * grad_dev; m_dev and v_dev are the moment arrays (zero before step 1). */
int mlp_adam_update(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                    uint32_t step, float lr, void *hip_stream);

/* ---------------------------------------------------------------- memory planning
 * The compression ratio decides how much device memory a circuit needs and
 * cannot be known before compressing (Section 3 feasibility analysis); the
 * memory manager plans with the block predictor instead of the worst case
 * (Section 4.4 two-level memory management).
 *
 * Planning form of the predictor's inputs: a rollout can advance only a
 * block's size, so planning uses feature 0 and the size label as log2 of
 * stream bytes per amplitude (log2 bytes - b, which makes circuits of
 * different block sizes comparable), features 1..24 fixed at the values of
 * an all-zero block, and the stage features 25..31 as usual.
 * sv_plan_features / sv_plan_labels -- sv_block_features / sv_block_labels
 * in that form (training data for the planning predictor; same arguments).
 *
 * mlp_predict_bytes -- the planning predictor rolled over a whole circuit
 * from |0...0>: the planning features of the initial state (computed on the
 * device from its directory headers) are advanced stage by stage, each
 * stage's predicted size becoming the next stage's feature 0 and the plan's
 * stage features filling features 25..31.  bytes_host[s] (host, one per
 * stage) receives the predicted stream bytes of the state after stage s
 * (sum over blocks of 2^(prediction + b)), whose maximum is the circuit's
 * predicted peak.  params_dev: SV_MLP_NPARAM device floats.  work_dev:
 * device, 256-byte aligned, mlp_predict_work bytes.  At most 2^20 blocks
 * (SV_ERR_UNSUPPORTED).  Synchronises. */
int sv_plan_features(const sv_t *sv, const sv_plan_t *p, size_t stage, float *feats_dev);
int sv_plan_labels(const sv_t *sv, float *log2_bytes_dev, int32_t *mode_dev);
int mlp_predict_work(const sv_plan_t *p, uint64_t *bytes);
int mlp_predict_bytes(const float *params_dev, const sv_plan_t *p, void *work_dev, uint64_t work_bytes,
                      double *bytes_host, void *hip_stream);

/* sv_admit -- admission of circuits into one batch under a device budget
 * (host only).  Circuit i (configuration cfgs[i]) gets device pools of
 * pool_bytes_out[i] bytes: from its predicted peak stream bytes
 * peak_bytes[i] (record bodies = stream bytes less 8 bytes of headers per
 * chunk, times 1 + margin, plus the segment slack), capped at the worst case;
 * with peak_bytes NULL, the worst case (the method without a predictor).
 * arena_bytes_out[i] receives sv_mem_required of that configuration.
 * Circuits are taken in order and admitted (admit_out[i] = 1) while the sum
 * of admitted arenas stays within budget; a circuit that does not fit is
 * skipped and later ones are still tried.  A prediction that falls short is
 * caught when the stage runs: records go to the attached host pool, or the
 * stage reports SV_ERR_CAPACITY and the circuit is re-run with worst-case
 * pools; records never depend on the pool sizes.  Output pointers except
 * admit_out may be NULL. */
int sv_admit(const sv_config_t *cfgs, size_t count, const double *peak_bytes, double margin, uint64_t budget,
             uint8_t *admit_out, uint64_t *pool_bytes_out, uint64_t *arena_bytes_out);

#ifdef __cplusplus
}
#endif
#endif /* BMQ_H */
