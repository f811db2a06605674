// Internal declarations shared by the host runtime (bmq_runtime.cpp) and the
// gfx950 kernels (bmq_kernels.hip).  Plain data only: descriptors that the
// host planner fills and the kernels read, and the kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmq {

constexpr int kChunk = 64;                      // values per codec chunk (one wavefront)
constexpr int kMaxOpQubits = 10;                // qubit slots of an operation descriptor
constexpr int kMaxDiagQubits = 9;               // widest diagonal operation (2^9-entry LDS table)
constexpr int kMaxTile = 13;                    // largest on-chip tile, log2 amplitudes
constexpr uint64_t kDirZero = 0;                // directory: chunk is entirely zero
constexpr uint64_t kDirInvalid = ~0ull;         // directory: body lost to an overflow
constexpr uint64_t kDirOffsetMask = (1ull << 40) - 1;   // body offset bits of an entry
constexpr uint32_t kSlotBytes = 576;            // one canonical chunk record, worst case 560

enum OpType : int32_t { OP_DENSE = 0, OP_DIAG = 1 };
enum IoMode : int32_t { IO_COMPRESSED = 0, IO_SCRATCH = 1 };
enum Mode : uint32_t { M_ZERO = 0, M_LZ = 1, M_Q0 = 2, M_VERB = 3 };

// One fused operation.  Operation qubit j is bit j of the matrix / table
// index.  DENSE: 2^k x 2^k complex64 matrix, row major, every qubit inside
// the tile.  DIAG: 2^k complex64 phases; a qubit outside the tile (pos < 0)
// is constant over the tile and read from the tile's base index.
struct OpDesc {
    int32_t type;
    int32_t k;
    int32_t pos[kMaxOpQubits];   // tile position of operation qubit j, or -1
    int32_t gq[kMaxOpQubits];    // global qubit of operation qubit j
    uint32_t data;               // offset into the complex64 data array
    uint32_t pad;
};

// Per-launch device counters.  The device pool a pass writes is split into
// n_seg segments (workgroup i uses segment i mod n_seg), each with its own
// cursor and statistics, so that no single address takes every workgroup's
// atomics.  A wave whose segment is full spills its bodies to the host pool
// (second memory level) through one cursor, C_HOST_CURSOR of segment 0.
// A launch's counter block is kSegments x C_NUM words.  The statistics cost
// a wave device-wide atomics only where the common case needs none: the
// bytes a segment holds on the device are its cursor less C_SPILLED (bytes
// of waves that found the segment full), C_MODE0 counts ZERO planes,
// C_MODE0 + 2 packs the Q0 | VERBATIM counts (32 bits each), and the LZ
// count is the rest of the pass's 2^(n-5) planes.
enum Counter : int {
    C_CURSOR = 0, C_OVERFLOW = 1, C_ZERO_CHUNKS = 2, C_MODE0 = 3, C_SPILLED = 4, C_HOST_BYTES = 6,
    C_HOST_CURSOR = 7, C_NUM = 8
};
constexpr int kSegments = 256;
constexpr uint32_t kMaxBodyBytes = 552;         // two planes, worst case

// Codec parameters: quantization step delta = 2^-s (the largest power of two
// <= 2 eb), scale = 2^s, eb as float32; code_ok is false when the step cannot
// code values at all (every chunk then stays VERBATIM).
struct CodecParams {
    int32_t domain;
    int32_t s;
    float ebf, delta, scale;
    int32_t code_ok;
};

// Where the record bodies of one state copy live: directory offsets below
// cap address the device pool, offsets cap + h address byte h of the host
// pool (pinned host memory the device reads and writes directly).
struct PoolView {
    const uint8_t *dev;
    const uint8_t *host;
    uint64_t cap;
};

struct PassArgs {
    int32_t n, t;
    int32_t tileq[16];        // tile position -> global qubit (positions 0..5 are qubits 0..5)
    int32_t nontile[48];      // non-tile qubits of the launch, ascending; tile id bit i -> qubit nontile[i]
    int32_t n_nontile;
    uint64_t fixed;           // bits of the amplitude index fixed for the whole launch (a group's outer bits)
    // scratch-plane positions of the same qubits: the scratch holds one group
    // of a multi-pass stage, with the group's qubits packed in ascending order
    // (identical to tileq / nontile when it holds the whole state)
    int32_t stileq[16];
    int32_t snontile[48];
    // the directories are indexed by the packed (scratch) positions as well:
    // a group staged on its own, with a directory of the group's chunks only
    int32_t dir_packed;
    int32_t op_begin, op_end;
    int32_t in_mode, out_mode;
    CodecParams cp;
    const uint64_t *dir_in;
    const uint8_t *pool_in;
    const uint8_t *host_in;
    uint64_t *dir_out;
    uint8_t *pool_out;
    uint8_t *host_out;
    uint64_t pool_cap;              // device pool bytes (offsets at and above go to the host pool)
    uint64_t host_cap;              // host pool bytes per state copy (0: no host level)
    uint64_t seg_cap;               // bytes per output pool segment
    int32_t n_seg;                  // segments in use (power of two <= kSegments)
    uint32_t seg_base;              // wave index of the launch's first wave (a group's launches continue the count)
    unsigned long long *counters;   // this stage's block of kSegments x C_NUM
    float *scr_re, *scr_im;
    const OpDesc *ops;
    const float2 *opdata;
    float *dump_re, *dump_im;       // test hook: values before encoding (or NULL)
    float *dumpd_re, *dumpd_im;     // test hook: values after decoding (or NULL)
    uint64_t dump_lo, dump_n;       // amplitudes [dump_lo, dump_lo + dump_n) are dumped
    int32_t mfma;                   // dense 4- and 5-qubit operations on the matrix cores
};

// ---- launch wrappers (bmq_kernels.hip) ----
hipError_t launch_pass(const PassArgs &a, hipStream_t s);
// first_block_dev[i]: first block of state i (ascending, first_block_dev[0] = 0);
// blocks: the total; every state in the launch uses tile size t and codec domain
hipError_t launch_pass_batch(int t, int domain, const PassArgs *args_dev, const uint32_t *first_block_dev, int n,
                             uint32_t blocks, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_check_dir(const uint64_t *dir, uint64_t n, uint64_t pool_cap, uint64_t host_cap, int domain,
                            unsigned long long *bad, hipStream_t s);

// Whole-circuit launch over a queue of (pass, tile) items, one workgroup per
// item.  Pass L owns items [first_item[L], first_item[L + 1]) (its tiles in
// order); dep[L] is the pass whose items must all be done before any item of
// L starts (-1: none), and dep[L] < L.  sync (device, zeroed before the
// launch): [0] next item, [1] abort flag, [2..3] unused, [4 + L] items of
// pass L done.
struct PersistArgs {
    const PassArgs *args;
    const uint32_t *first_item;
    const uint32_t *tiles_per_item;
    const int32_t *dep;
    uint32_t *sync;
    uint64_t limit_ticks;       // longest wait, in s_memrealtime ticks
    uint32_t n_pass, total, max_grid;
    int32_t system_scope;       // records may live in host memory
};
constexpr int kSyncHead = 4;
hipError_t launch_pass_queue(int t, int domain, const PersistArgs &pa, hipStream_t s);
hipError_t launch_init_state(uint64_t *dir, uint64_t n_chunks, uint8_t *pool,
                             unsigned long long *counters, CodecParams cp, hipStream_t s);
hipError_t launch_export(const uint64_t *dir, const PoolView &pv, CodecParams cp,
                         uint64_t chunk0, uint64_t n_chunks, float2 *dst, hipStream_t s);
hipError_t launch_amplitudes(const uint64_t *dir, const PoolView &pv, CodecParams cp,
                             const uint64_t *idx, uint64_t k, uint64_t n_chunks, float2 *dst,
                             hipStream_t s);
// Reference of an FP64 reduction: none, a complex128 device array (element 0
// = the first amplitude of the reduced range), or a second compressed state.
enum { REF_NONE = 0, REF_C128 = 1, REF_STATE = 2 };
struct RefView {
    int32_t kind;
    const double2 *c128;
    const uint64_t *dir;
    PoolView pv;
    CodecParams cp;
};
// partials: n_partials x 5 doubles, accumulated into (zero them first)
hipError_t launch_fidelity_partial(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint64_t chunk0,
                                   uint64_t n_chunks, const RefView &rv, double *partials, int n_partials,
                                   hipStream_t s);
hipError_t launch_fidelity_final(const double *partials, int n_partials, double *out5, hipStream_t s);
// |psi|^2 per group of chunks_per_group chunks (a multiple of 16)
hipError_t launch_group_norm(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint32_t chunks_per_group,
                             uint64_t n_groups, double *gnorm, hipStream_t s);
hipError_t launch_sample(const uint64_t *dir, const PoolView &pv, CodecParams cp, uint32_t chunks_per_group,
                         const uint32_t *grp, const double *resid, uint64_t k, uint64_t *out, hipStream_t s);
// the 7 stage features of the block predictor (features 25..31)
struct StageFeats {
    float v[7];
};
// feats: n_blocks x 32 (or NULL); label_bytes / label_mode: n_blocks each
// (both or neither); n_blocks < 2^31
hipError_t launch_block_stats(const uint64_t *dir, uint64_t chunks_per_block, uint64_t n_blocks,
                              const StageFeats &sf, float *feats, float *label_bytes,
                              int32_t *label_mode, hipStream_t s);
// stand-alone codec on whole chunks: slot form (record i at slots + i kSlotBytes)
hipError_t launch_codec_slots_encode(const float *re, const float *im, uint64_t nch, CodecParams cp,
                                     uint8_t *slots, uint32_t *sizes, hipStream_t s);
hipError_t launch_codec_slots_decode(const uint8_t *slots, uint64_t nch, CodecParams cp, float *re, float *im,
                                     hipStream_t s);
// stream form: sizes (nch u32) and off (nch + 1 u64) are scratch; nothing is
// written to dst when 16 + total > cap (off[nch] = total record bytes)
hipError_t launch_codec_stream_encode(const float *re, const float *im, uint64_t nch, CodecParams cp,
                                      uint32_t *sizes, uint64_t *off, uint8_t *dst, uint64_t cap, uint32_t ebbits,
                                      hipStream_t s);
// record offsets of a stream (off: nch u64); *bad set on a malformed stream
hipError_t launch_codec_stream_decode(const uint8_t *src, uint64_t bytes, uint64_t nch, CodecParams cp,
                                      uint64_t *off, uint32_t *bad, hipStream_t s);
hipError_t launch_codec_read(const uint8_t *src, const uint64_t *off, uint64_t nch, CodecParams cp, float *re,
                             float *im, hipStream_t s);

// ---- host-resident pipeline: staging of one SV group on the device ----
// Add the body offset of each staged block to its chunks' directory entries
// (entries of all-zero chunks stay 0): entry i belongs to block
// i / chunks_per_block, whose bodies start at body_off[block] of the staging
// pool.
hipError_t launch_rebase_dir(uint64_t *dir, uint64_t n_entries, uint32_t chunks_per_block, const uint64_t *body_off,
                             hipStream_t s);
// Pack a staged group's output (directory dir in packed chunk order, bodies
// in pool) into one image per SV block: [the block's directory, offsets
// relative to the image's body area] [its bodies in chunk order].  Three
// steps over segments of seg = min(1024, chunks_per_block) chunks:
//   sizes:   rel[i] = body offset of chunk i within its segment, segsum[k] =
//            body bytes of segment k;
//   offsets: segsum scanned in place to each segment's offset within its
//            block; img_off[j] = offset of block j's image (j <= n_blocks, the
//            last entry the total; images are 16-byte aligned) and
//            img_off[n_blocks + 1 + j] = block j's body bytes;
//   write:   every image's directory and bodies into img.
hipError_t launch_pack_sizes(const uint64_t *dir, uint64_t n_chunks, uint32_t seg, uint32_t *rel, uint64_t *segsum,
                             hipStream_t s);
hipError_t launch_pack_offsets(uint64_t *segsum, uint32_t chunks_per_block, uint32_t seg, uint32_t n_blocks,
                               uint64_t *img_off, hipStream_t s);
hipError_t launch_pack_write(const uint64_t *dir, const uint8_t *pool, uint32_t chunks_per_block, uint32_t seg,
                             uint64_t n_chunks, const uint32_t *rel, const uint64_t *segsum, const uint64_t *img_off,
                             uint8_t *img, hipStream_t s);

// static device scratch of the allocation-free codec entry point: holds the
// codec workspace (record sizes, offsets) of up to kNoAllocMaxValues values
constexpr uint64_t kNoAllocMaxValues = 1ull << 24;
constexpr uint64_t kNoAllocScratchBytes = 4ull << 20;
constexpr int kMaxDevices = 64;
// device address of that scratch on the current device (looked up once per device)
hipError_t noalloc_scratch(void **ptr);

// ---- block predictor (bmq_mlp.hip) ----
uint64_t mlp_work_floats(uint32_t batch);
hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t batch, float *out, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float *P, const float *X, const float *y_bytes, const int32_t *y_mode,
                                uint32_t batch, float *work, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *P, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t s);
// rows 2.. of X (n_blocks x 32) <- row 1
hipError_t launch_replicate_rows(float *X, uint32_t n_blocks, hipStream_t s);
// *total <- sum of 2^(out0 + b) over the blocks; X's feature 0 <- out0, features 25..31 <- next
hipError_t launch_rollout_step(float *X, const float *out, uint32_t n_blocks, const StageFeats &next, int b,
                               double *total, hipStream_t s);
// planning form of features (X, may be NULL) and size labels (y, may be NULL)
hipError_t launch_plan_form(float *X, float *y, uint32_t n_blocks, int b, hipStream_t s);

}  // namespace bmq
