// Internal declarations shared by the HIP kernels and the C ABI of libwrls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wrls {

constexpr int kMaxD = 10;
// Pixels per chunk of the state layout (below); a state copy holds a whole
// number of chunks, and the second copy of a stream starts this many floats
// (256 bytes) past the end of the first.
constexpr size_t kPlaneAlign = 64;

__host__ __device__ constexpr int packed_floats(int d) { return d * (d + 1) / 2; }
__host__ __device__ constexpr int state_floats(int d) { return packed_floats(d) + 3 * d; }

// Position of P(i, m), i <= m, in the packed upper triangle, row-major.
__host__ __device__ constexpr int packed_index(int d, int i, int m)
{
    return i * d - (i * (i - 1)) / 2 + (m - i);
}

// State layout of one copy (S entries per pixel, `pitch` pixel slots, a
// multiple of 64): pixels are grouped in chunks of 64 consecutive pixel
// indices, and each chunk holds all S entries of its pixels contiguously
// (S * 256 bytes).  Inside a chunk, the first 4 * (S / 4) entries form S / 4
// groups of 16-byte vectors -- entry k of pixel l at group k / 4, vector l,
// element k % 4, so one 128-bit access moves four entries of a pixel and a
// wave's access to one group covers 1 KiB of consecutive bytes -- followed by
// the remaining S % 4 entries as groups of 4-byte scalars.  The copy is
// S * pitch floats.
__host__ __device__ constexpr int vec_planes(int S) { return S / 4; }
// Byte offset of pixel j's 16-byte slot (vector entries) and 4-byte slot
// (scalar entries) relative to the start of an entry group of its chunk.
__host__ __device__ inline uint32_t vslot(uint32_t j, int S)
{
    return (j >> 6) * (uint32_t)S * 256u + (j & 63u) * 16u;
}
__host__ __device__ inline uint32_t sslot(uint32_t j, int S)
{
    return (j >> 6) * (uint32_t)S * 256u + (j & 63u) * 4u;
}
// Byte offset, within a chunk, of vector group g and of scalar entry
// 4 * (S / 4) + r.
__host__ __device__ inline uint32_t vgroup(int g) { return (uint32_t)g * 1024u; }
__host__ __device__ inline uint32_t sgroup(int S, int r)
{
    return (uint32_t)vec_planes(S) * 1024u + (uint32_t)r * 256u;
}
// Order of a pixel's entries in the state: beta (3 rows of d, the colour
// channel's coefficients contiguous), then the packed P, then the paper-mode
// history.  With beta first, channel c starts at entry c * d: at d = 4 and 8
// every channel starts on a 16-byte vector, so the spatial blend reads a
// channel's coefficients with the fewest vector loads.  The export and import
// order (wrls_get_state / wrls_set_state) is P, then beta, then the history.
__host__ __device__ constexpr int beta_entry0(int) { return 0; }
__host__ __device__ constexpr int p_entry0(int d) { return 3 * d; }
// Position in the state of export-order entry k.
__host__ __device__ inline int state_entry_index(int d, int k)
{
    const int np = packed_floats(d);
    return k < np ? p_entry0(d) + k : (k < np + 3 * d ? beta_entry0(d) + (k - np) : k);
}
// Byte offsets of export-order entry k of pixel j: a per-pixel part (voff)
// and a per-entry part (soff); the entry's address is base + soff + voff.
__host__ __device__ inline void entry_offsets(int S, int d, int k_export, uint32_t j,
                                              uint32_t &voff, uint32_t &soff)
{
    const int G = vec_planes(S);
    const int k = state_entry_index(d, k_export);
    if (k < 4 * G) {
        voff = vslot(j, S) + (uint32_t)(k % 4) * 4u;
        soff = vgroup(k / 4);
    } else {
        voff = sslot(j, S);
        soff = sgroup(S, k - 4 * G);
    }
}

// Everything one launch of the per-frame kernel needs for one image.
struct FrameArgs {
    const void *color;      // [3][H][W] float or _Float16
    const void *feats;      // [d-1][H][W] float or _Float16
    const float *var;       // [H][W] or null (unit weights)
    const float *motion;    // [2][H][W] or null (zero motion)
    float *out;             // [3][H][W]
    const float *state_in;  // state copy of the previous frame (layout above)
    float *state_out;       // state copy of this frame
    int32_t W, H;
    int64_t pitch;          // pixel slots of a state copy (layout above)
    float lambda, inv_lambda, p0, var_floor;
    float alpha, inv_h2, eps;  // paper mode: Eq. 12 history weight, 1/h^2 and eps of Eq. 13
    float inv_sigma0;       // automatic forgetting factor: 1 / the prescribed information
    float lambda_min;       // automatic forgetting factor: lower limit (lambda is the upper)
    int32_t auto_lambda;    // 1: forgetting factor chosen per pixel and step
    int32_t fresh;          // 1: no history (first frame)
    int32_t unit_weight;    // 1: w = 1 (plain RLS)
    int32_t nearest;        // 1: nearest reprojection
    int32_t tiles_x;        // tiles per image row
    int32_t tiles_y;        // tile rows
    int32_t strip_w;        // tiles per vertical strip of the tile order
};

// Launch shape of the per-frame kernel: a tile is (1 << tw_log2) pixels
// wide and block_threads >> tw_log2 rows high; one thread per pixel.  Tiles
// run in vertical strips of strip_w tiles (0: one strip, the full width).
struct TileShape {
    int32_t tw_log2;
    int32_t block_threads;
    int32_t strip_w;
};


// Device-resident description of one batched step (rewritten every step):
// the frames of up to kMaxBatch streams, all with the same d and input type
// and one tile shape, and the prefix sums of their tile counts.
constexpr int kMaxBatch = 64;
struct BatchTable {
    int32_t n;                  // frames in this step
    int32_t total_tiles;        // prefix[n]
    TileShape tile;             // strip_w unused: each image runs row by row
    int32_t prefix[kMaxBatch + 1];
    FrameArgs frame[kMaxBatch];
};

// Everything one launch of the spatial blend needs (Sec. 5.3, last
// paragraph): the current state, the frame's predictor source, the step's
// output as the range guide, and the output.
struct BlendArgs {
    const float *state;     // current state copy (layout above)
    const void *feats;      // [d-1][H][W] float or _Float16 (null in paper mode or d = 1)
    const float *guide;     // [3][H][W] output of the step (temporal prediction)
    float *out;             // [3][H][W]
    int32_t W, H;
    int64_t pitch;
    float inv2ss, inv2sr;   // 1/(2 sigma_s^2), 1/(2 sigma_r^2); 0 turns a factor off
    int32_t tiles_x;        // blend tiles per image row
    int32_t tiles_y;
    int32_t strip_w;        // tiles per vertical strip of the tile order (launch_blend sets it)
};
// Blend tile: kBlendTW x kBlendTH output pixels per workgroup of
// kBlendTW * kBlendTH / kBlendRPT threads (each thread computes kBlendRPT
// vertically adjacent pixels), window radius kBlendR.
constexpr int kBlendTW = 64;
constexpr int kBlendRPT = 2;
constexpr int kBlendTH = 4 * kBlendRPT;
constexpr int kBlendR = 2;

// Checked builds (compiled with WRLS_CHECKED: libwrls_checked.so): the
// kernels test every gathered tap, every 16-byte state access and every LDS
// index against its array before use, skip a failing access and record its
// site.  Sites, one flag each:
enum CheckSite {
    kChkGatherTap = 0,  // a reprojection tap outside the image or the state copy
    kChkStateStore,     // a pixel's state or output store outside its arrays
    kChkBlendHalo,      // a blend halo load outside the state copy
    kChkBlendLds,       // a blend LDS index outside the staged tile
    kChkPaperLds,       // a paper-mode 3x3 LDS index outside the staged tile
    kChkBatchFrame,     // a batched tile mapped to no frame of the table
    kNumCheckSites
};
// Copies the per-site flags of this device into flags[kNumCheckSites] and
// clears them (synchronises the device).  hipErrorNotSupported in builds
// without checks.
hipError_t read_and_clear_checks(uint32_t *flags);
// Raises the flags of the sites in mask from a kernel (checked builds).
hipError_t raise_checks(uint32_t mask, hipStream_t st);

// S: state entries per pixel (state_floats(d), plus 3 history entries in
// paper mode).
hipError_t launch_reset(float *state, int64_t npix, int d, int S, float p0, hipStream_t st);
// Copies export-order entries k0 .. k0 + count - 1 of every pixel between a
// state copy (layout above) and caller planes [count][npix]; to_state
// selects the direction.
hipError_t launch_convert(float *state, float *planes, int64_t npix, int d, int S, int k0,
                          int count, bool to_state, hipStream_t st);
hipError_t launch_step(int d, bool f16, const FrameArgs &a, TileShape ts, hipStream_t st);
// The step's loads and stores without reprojection or arithmetic (a
// measurement reference): a's state_in is moved unchanged to state_out.
hipError_t launch_probe(int d, bool f16, bool paper, const FrameArgs &a, TileShape ts,
                        hipStream_t st);
// n16 16-byte vectors from src to dst (16-byte loads, non-temporal stores).
hipError_t launch_copy(void *dst, const void *src, size_t n16, hipStream_t st);
// The paper's own predictor and weight (d = 4, state with history).
hipError_t launch_step_paper(bool f16, const FrameArgs &a, TileShape ts, hipStream_t st);
// The 5x5 spatial blend of neighbour-model predictions; paper: p = [1, z]
// from the state's history entries (d = 4).
hipError_t launch_blend(int d, bool f16, bool paper, const BlendArgs &a, hipStream_t st);
// One persistent launch of `grid` workgroups of tab->tile.block_threads
// threads over every tile of every frame in the device table `tab`.
hipError_t launch_step_batched(int d, bool f16, const BatchTable *tab, int32_t grid,
                               int32_t block_threads, hipStream_t st);
// Steps that allocate nothing: the device address of this device's fixed
// frame table (looked up once per device), and the launches that write a
// host-built table into it (kernel arguments carry the table; no copy).
hipError_t noalloc_table(BatchTable **tab);
hipError_t launch_fill_table(BatchTable *tab, const BatchTable &host, hipStream_t st);
// The batched kernel's entry point (for graph kernel nodes); null for a bad d.
const void *batched_kernel_fn(int d, bool f16);
// Workgroups of block_threads threads of the batched kernel that fit on one
// compute unit at once.
hipError_t batched_blocks_per_cu(int d, bool f16, int32_t block_threads, int *blocks_per_cu);

}  // namespace wrls
