// Batched-state path on the gfx950 matrix cores.
//
// For B domain states of one network, the support counts of one step of
// Eq. (1) are products of the 0/1 relation matrix R[(x,a),(y,b)] (int8) with
// the domain matrix Dom[(y,b), s] (int8): for a constrained pair (x,y),
// count(x,a,y,s) = sum_b R[x,a,y,b] * Dom[y,b,s] (tensorRevise of
// Algorithm 1; at most d <= 32, so int32 accumulation is exact). Unlike a
// plain GEMM, the counts of different neighbours y are not summed: a value
// survives only if every neighbour's count is non-zero (Algorithm 1 clamps
// the counts and tests that the clamped sum equals the number of neighbours).
// The kernel turns each count into a zero flag inside the matrix-core
// accumulator (two arcs per accumulator chain, see kBias below) and ORs the
// flags over y.
//
// Tiling. A workgroup of 8 waves owns 16 variables x (a pair per wave) and
// 128 states (4 sub-tiles of 32). It walks y = 0..n-1 in blocks of 8, two
// blocks (a superblock) per stage of a 2-stage LDS buffer. The domain bytes
// of a block for its 128 states (stored per variable in the order of the
// active-state slots, so one (y, half) row of 128 slots is 2 KiB of
// consecutive memory) are loaded into registers one superblock ahead and
// written to the other stage at the end of the block;
// each wave loads its pair's relation operands for the block's neighbours
// (packed once per network, see mfma_pack_ops_kernel) into registers, also a
// block ahead, and multiplies them with the staged bytes, one
// v_mfma_i32_32x32x32_i8 per (operand, sub-tile). Workgroups of one x-tile
// are placed on one XCD so that the operands they share meet in that XCD's
// L2.
//
// Steps. Each step writes the new domain bytes (double buffer), and per
// (variable, slot word of 32 states) a change mask and a wipe-out mask. A
// reduce kernel folds those masks over the variables per state; a one-block
// finalise kernel applies Algorithm 1's loop test per state and compacts the
// states that go on into the next step's active list; a gather kernel moves
// their domain bytes to their new slots. A step with too few active states to
// fill the chip splits every tile's neighbour blocks over several workgroups
// (mfma_split_finish_kernel applies their flags).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rac_mfma.h"

namespace rac {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kMW = 8;            // waves per workgroup
constexpr int kXW = 2;            // variables per wave
constexpr int kMX = kMW * kXW;    // variables per workgroup
constexpr int kMSub = 4;          // 32-state sub-tiles per wave
constexpr int kMS = 32 * kMSub;   // states per workgroup
constexpr int kMY = 8;            // neighbours per LDS block
constexpr int kSB = 2;            // neighbour blocks per LDS stage (a superblock)
constexpr int kMThreads = 64 * kMW;
constexpr int kMaxTrackedSteps = 256;   // steps whose re-examined arcs are counted
constexpr int kNsegMax = 4;             // workgroups per tile of a split step, at most

// 4 bits -> 4 bytes holding 0/1 (bit i of v becomes byte i). The factor places
// copies of v 7 bits apart, so no two copies overlap and no carry occurs.
__device__ __forceinline__ uint32_t spread4(uint32_t v) { return (v * 0x00204081u) & 0x01010101u; }

struct MState {
    long long checks;     // support checks so far
    unsigned long long degsum;
    int32_t changed;      // the current step changed this state
    int32_t wiped;        // some domain is empty (sticky)
    int32_t iters, status, rc, done;
};

struct MArgs {
    int32_t n, d, capB;               // capB: state slots of the domain buffers
    const int32_t *deg;               // [n]
    const v4i *aop;                   // [operands][64 lanes] matrix-core A operands, 16 bytes
                                      // per lane (see mfma_pack_ops_kernel)
    const uint32_t *udesc;            // [pairs][nblk] units of pair p in neighbour block b:
                                      // bits 3u..3u+2: block slot (y - 8b) of unit u; bits
                                      // 24-26: chained pairs nc; 27-30: shared neighbours nb;
                                      // bit 31: leftover kind (0: of x0, 1: of x1)
    const uint32_t *ubase;            // [pairs][nblk] first operand (bits 0-26) and unit count
                                      // nu (bits 27-31) of pair p in block b
    int32_t nblk;                     // ceil(n / 8)
    int8_t *dom8[2];                  // [n][2][capB][16]: bytes 16h .. 16h+15 of the domain as
                                      // bytes 0 / -1 (0xFF: value present)
                                      // of (x, state slot); [0]: the current step's input,
                                      // [1]: its output (same slot order)
    uint32_t *chg, *wipe;             // [n][words]
    uint32_t *kill;                   // [n][capB] values of (x, slot) left without support by
                                      // a split step (bit a), zero between steps
    int32_t words;                    // capB / 32
    int32_t *act[2];                  // active state lists (by step parity)
    int32_t *prev_slot[2];            // slot each listed state had in the previous step
    int32_t *slot_map;                // [capB] old slot -> new slot, or -1 when the state stopped
    int32_t *cnt;                     // [2] active counts
    MState *st;                       // [capB]
    uint32_t *ych;                    // [capB/128][nw32]: bit y of tile t's words is set iff
                                      // variable y changed in the previous step in some state
                                      // of state tile t (Proposition 2)
    int32_t nw32;                     // ceil(n / 32)
    int32_t skip;                     // 1: steps k >= 2 skip neighbours no state of the tile changed
    unsigned long long *stepops;      // [kMaxTrackedSteps + 2] arcs re-examined by the states of
                                      // step k (sum over states of deg of the changed variables)
    int32_t *ctl;                     // [4] device control of the step loop: [0] 1 once the
                                      // matrix-core steps are over, [1] the last step they ran,
                                      // [2 + (k & 1)] workgroups per tile of step k (split)
    int32_t handoff;                  // stop when at most this many states remain (0: never)
    int32_t cus, force_seg, ntiles_x; // compute units; forced split (0: none); x-tiles
    int32_t mode, max_sweeps, B, xcd_map;
    long long checks1;                // support checks of step 1: 2m * d * d
    const uint64_t *din;              // [B][n]
    uint64_t *dout;                   // [B][n] (written as states stop)
    int32_t *iters_out, *status_out, *rc_out;
    long long *checks_out;
};

// Byte offset of the 16 domain bytes (x, half h, slot) in a domain buffer.
__device__ __forceinline__ int64_t dom_off(const MArgs &A, int32_t x, int h, int32_t slot) {
    return (((int64_t)x * 2 + h) * A.capB + slot) * 16;
}

// The step loop runs on the device: every kernel of step k returns at once
// when the matrix-core steps ended before step k (the host enqueues whole
// rounds of steps and reads the control words once per round).
__device__ __forceinline__ bool step_off(const MArgs &A, int k) {
    return A.ctl[0] != 0 && k > A.ctl[1];
}

// Workgroups per tile for a step with `active` states: enough tiles to fill
// the compute units, at most 4 (or the forced count).
__device__ __forceinline__ int split_for(const MArgs &A, int active) {
    const int sact = (active + kMS - 1) / kMS;
    const int tiles = A.ntiles_x * sact;
    const int nsb = (A.nblk + kSB - 1) / kSB;   // superblocks (the unit of a split)
    const int cap = nsb < kNsegMax ? nsb : kNsegMax;
    if (A.force_seg > 0) return A.force_seg < cap ? A.force_seg : cap;
    int sg = tiles > 0 ? A.cus / tiles : 1;
    // workgroups the grid holds for each active tile: those of the idle tiles
    const int avail = sact > 0 ? (A.words * 32 / kMS) / sact : 1;
    sg = sg < avail ? sg : avail;
    return sg < 1 ? 1 : (sg > cap ? cap : sg);
}

// 32 domain bytes (two 16-byte halves, 0 or 0xFF) -> bit mask, and back.
__device__ __forceinline__ uint64_t bytes_to_mask(const uint4 lo, const uint4 hi) {
    const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint64_t m = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if ((w[q] >> (8 * t)) & 0xFFu) m |= 1ull << (4 * q + t);
    return m;
}
__device__ __forceinline__ void mask_to_bytes(uint64_t m, uint4 &lo, uint4 &hi) {
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = spread4((uint32_t)(m >> (4 * q)) & 0xFu) * 0xFFu;
    lo = make_uint4(w[0], w[1], w[2], w[3]);
    hi = make_uint4(w[4], w[5], w[6], w[7]);
}

// ---------------------------------------------------------------------------

__global__ void mfma_init_kernel(MArgs A) {
    const int64_t total = (int64_t)A.B * A.n;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < total; i += nth) {
        const int32_t x = (int32_t)(i / A.B);
        const int32_t s = (int32_t)(i - (int64_t)x * A.B);   // slot = state in step 1
        uint4 lo, hi;
        mask_to_bytes(A.din[(int64_t)s * A.n + x], lo, hi);
        *reinterpret_cast<uint4 *>(A.dom8[0] + dom_off(A, x, 0, s)) = lo;
        *reinterpret_cast<uint4 *>(A.dom8[0] + dom_off(A, x, 1, s)) = hi;
    }
    for (int64_t s = tid; s < A.B; s += nth) {
        MState &m = A.st[s];
        m.checks = A.checks1;
        m.degsum = 0;
        m.changed = 0;
        m.wiped = 0;
        m.iters = 0;
        m.status = 0;
        m.rc = 0;
        m.done = 0;
        A.act[0][s] = (int32_t)s;
    }
    if (tid == 0) {
        A.cnt[0] = A.B;
        A.cnt[1] = 0;
        A.ctl[0] = 0;
        A.ctl[1] = 0;
        A.ctl[2 + 1] = split_for(A, A.B);   // step 1
        if (A.rc_out) *A.rc_out = 0;
    }
}


constexpr int kStages = 2;                          // LDS stages (double buffer)
constexpr int kBTile = kMY * 2 * kMS;               // v4i per block's domain tile (32 KiB)
constexpr int kMaxUnits = kMY;                      // operands of a pair in one block: <= 8
constexpr size_t kMSmem = (size_t)kStages * kSB * kBTile * 16;   // 128 KiB
constexpr int kRowsPerWave = kMY * 2 / kMW;         // domain rows (y, half) each wave copies
constexpr int kParts = kMS / 64;                     // 64-slot parts of a row
constexpr int kCopyPerBlock = kRowsPerWave * kParts; // 16-byte copies per lane and block
static_assert(kMY * 2 % kMW == 0 && kMS % 64 == 0, "the tile copy splits evenly over the waves");
constexpr int kTabShift = 6;                        // lane tables cover 64 blocks

// Zero-count flags. Domain bytes are 0 or -1 (0xFF). A wave owns the pair of
// variables x0 = 2p, x1 = 2p+1 and walks the neighbours y of either in blocks
// of 8. For one matrix-core product D = kBias + A . Dom(y) with the operand
//   A[a][b] = R(x0,y)[a][b] + 64 R(x1,y)[a][b]   (bytes 0, 1, 64, 65),
// every (value a, state) gets D = -2016 - c0 - 64 c1 = ~((c0 + 31) + 64 (c1 + 31)),
// c0 and c1 <= 32 being the support counts of (x0, a) and (x1, a) on y: the
// two 6-bit fields c + 31 do not carry into each other and have bit 5 set iff
// c > 0, so bit 5 (bit 11) of D is set iff (x0, a) ((x1, a)) has no support
// on y. The kernel ORs these words over all neighbours: a value survives iff
// its flag stays clear (Eq. (1): it needs a support on every constraint).
//
// A neighbour of both variables costs one product for two arcs. A neighbour
// of only x0 (operand R(x0,y)) and one of only x1 (operand 64 R(x1,y)) of the
// same block are chained into one accumulator, so both fields are again
// real counts. For a neighbour left over (the block has more of one kind than
// of the other) only the flag of its own variable is OR-ed in. The units of a
// block are stored chains first, then shared neighbours, then leftovers, so
// that every kind starts at a known unit index.
constexpr int kBias = -2016;
constexpr int kFlag0 = 1 << 5, kFlag1 = 1 << 11;
static_assert(kXW == 2, "the zero-count flags pack exactly two variables per word");

__device__ __forceinline__ v16i mfma8(const v4i a, const v4i b, const v16i c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// nseg > 1 splits the neighbour blocks of every (x-tile, state tile) over
// nseg workgroups (for steps with few active states, so that the grid still
// fills the chip); each ORs its flags into A.kill and mfma_split_finish_kernel
// applies them.
__global__ __launch_bounds__(kMThreads) void mfma_sweep_kernel(MArgs A, int k, int fgrid) {
    extern __shared__ v4i s_lds[];   // kStages domain tiles [kMY][2][kMS]
    if (step_off(A, k)) return;
    const int nact = A.cnt[(k - 1) & 1];
    const int nseg = A.ctl[2 + (k & 1)];   // workgroups per tile this step
    // The grid holds fgrid workgroups per (x-tile, state tile) of the whole
    // batch; a step uses the first nseg x (tiles of its active states) of
    // them, so that a step with few states splits each tile's neighbour
    // blocks over workgroups the idle state tiles leave. Workgroup ->
    // (x-tile, state tile, segment): the state tiles of one x-tile share
    // blockIdx % 8 and so an XCD.
    const int sact = (nact + kMS - 1) / kMS;   // active state tiles
    int xt, stile, seg, i;
    if (A.xcd_map) {
        i = blockIdx.x >> 3;
        const int t = i / nseg;
        seg = i - t * nseg;
        stile = t % sact;
        xt = (t / sact) * 8 + (blockIdx.x & 7);
    } else {
        i = blockIdx.x;
        const int t = i / nseg;
        seg = i - t * nseg;
        stile = t % sact;
        xt = t / sact;
    }
    (void)fgrid;
    const int st0 = stile * kMS;
    if (sact == 0 || xt * kMX >= A.n) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // this workgroup's superblocks [sblo, sbhi) of kSB neighbour blocks (all
    // of them unless split), which end at block bhi
    const int nsb = (A.nblk + kSB - 1) / kSB;
    const int sblo = (int)((int64_t)seg * nsb / nseg), sbhi = (int)((int64_t)(seg + 1) * nsb / nseg);
    const int bhi = sbhi * kSB < A.nblk ? sbhi * kSB : A.nblk;
    // this wave's pair p and its variables x = 2p + i
    const int pr = xt * kMW + wave;
    int xs[kXW];
    bool xvs[kXW];
#pragma unroll
    for (int i = 0; i < kXW; ++i) {
        xs[i] = kXW * pr + i;
        xvs[i] = xs[i] < A.n;                       // wave-uniform
    }
    const bool pv = xvs[0];
    const int8_t *din = A.dom8[0];
    const int half = lane >> 5, col = lane & 31;
    const bool skip_on = A.skip && k > 1;

    // Lane tables of a chunk of 64 blocks: lane l holds the unit descriptor
    // and the first operand / unit count of block 64c + l. One copy follows
    // the blocks whose operands are being loaded (one ahead), one the block
    // being multiplied.
    uint32_t tdI = 0, tbI = 0, tdC = 0, tbC = 0;
    int chunkI = -1;
    auto load_tab = [&](int c) {
        const int b = (c << kTabShift) + lane;
        const bool ok = pv && b < A.nblk;
        const int64_t o = (int64_t)(ok ? pr : 0) * A.nblk + (ok ? b : 0);
        const uint32_t dsc = A.udesc[o], bs = A.ubase[o];
        tdI = ok ? dsc : 0u;
        tbI = ok ? bs : 0u;
    };
    // Proposition 2: after step 1 the workgroup visits only the superblocks
    // with a neighbour that changed in the previous step in some state of its
    // state tile. Bit i of mask_of(c) is set iff block 64c + i has such a
    // neighbour
    // (lanes 0..15 read the tile's change words of the chunk, 32 variables
    // = 4 blocks each). Every wave computes the same blocks, so the
    // workgroup's barriers match.
    auto mask_of = [&](int c) -> uint64_t {
        const int w = (c << (kTabShift - 2)) + lane;
        const bool okw = lane < (1 << (kTabShift - 2)) && w < A.nw32;
        const uint32_t yw = okw ? A.ych[(int64_t)stile * A.nw32 + w] : 0u;
        uint64_t m = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // bit l of b: block 4l + r of the chunk; spread to bit 4l + r
            uint64_t b = __ballot(((yw >> (8 * r)) & 0xFFu) != 0) & 0xFFFFull;
            b = (b | (b << 24)) & 0x000000FF000000FFull;
            b = (b | (b << 12)) & 0x000F000F000F000Full;
            b = (b | (b << 6)) & 0x0303030303030303ull;
            b = (b | (b << 3)) & 0x1111111111111111ull;
            m |= b << r;
        }
        return m;
    };
    int mchunk = -1;
    uint64_t mbits = 0;
    static_assert(kSB == 2 && (1 << kTabShift) % kSB == 0, "superblocks of two blocks, within a chunk");
    // the first superblock >= from in [sblo, sbhi) the workgroup visits, or sbhi
    auto next_sb = [&](int from) -> int {
        if (!skip_on) return from < sbhi ? from : sbhi;
        while (from < sbhi) {
            const int b0 = from * kSB, c = b0 >> kTabShift;
            if (c != mchunk) {
                mchunk = c;
                mbits = mask_of(c);
            }
            // bit 2i: superblock i of the chunk has a block to visit
            const uint64_t sm = (mbits | (mbits >> 1)) & 0x5555555555555555ull;
            const uint64_t m = sm & (~0ull << (b0 & 63));
            if (m) {
                const int sbn = ((c << kTabShift) + __builtin_ctzll(m)) / kSB;
                return sbn < sbhi ? sbn : sbhi;
            }
            from = ((c + 1) << kTabShift) / kSB;
        }
        return sbhi;
    };
    auto lane_word = [&](uint32_t t, int b) -> uint32_t {
        return (uint32_t)__builtin_amdgcn_readlane((int)t, b & 63);
    };

    // Operand table word (first operand, unit count) of block b; the copy
    // of the lane table that follows the operand loads moves to b's chunk.
    auto ops_word = [&](int b) -> uint32_t {
        if ((b >> kTabShift) != chunkI) {
            chunkI = b >> kTabShift;
            load_tab(chunkI);
        }
        return lane_word(tbI, b);
    };
    // Operands u0, u0+1 of the block whose table word is w, into Aop[u0],
    // Aop[u0+1] (16 bytes per lane each; units past the block's count load
    // its first operand again)
    v4i Aop[kMaxUnits];
    auto load_two = [&](uint32_t w, int u0) {
        const int nu = (int)(w >> 27);
        const v4i *src = A.aop + (int64_t)(w & 0x7FFFFFFu) * 64 + lane;
        Aop[u0] = src[(u0 < nu ? u0 : 0) * 64];
        Aop[u0 + 1] = src[(u0 + 1 < nu ? u0 + 1 : 0) * 64];
    };
    // The domain tile of block `blk`: 16 rows (neighbour yl, half h) of 128
    // consecutive slots, 2 KiB each in both memories; wave w copies rows 2w
    // and 2w+1 as 1 KiB halves, loaded into registers (fetch) and written to
    // block position sh of an LDS stage (store). A neighbour past n copies
    // variable n-1's row (never a neighbour of anything); slots past the
    // active ones are in the buffer and never used. (Registers rather than
    // direct-to-LDS copies: the compiler then waits for each operand load
    // precisely.)
    v4i cp[kCopyPerBlock];
    auto fetch = [&](int blk) {
#pragma unroll
        for (int i = 0; i < kCopyPerBlock; ++i) {
            const int row = wave * kRowsPerWave + i / kParts, part = i % kParts;
            const int yl = row >> 1, h = row & 1;
            int y = blk * kMY + yl;
            y = y < A.n ? y : A.n - 1;
            cp[i] = *reinterpret_cast<const v4i *>(din + dom_off(A, y, h, st0 + part * 64 + lane));
        }
    };
    auto store = [&](int stg, int sh) {
        v4i *bt = s_lds + (stg * kSB + sh) * kBTile;
#pragma unroll
        for (int i = 0; i < kCopyPerBlock; ++i) {
            const int row = wave * kRowsPerWave + i / kParts, part = i % kParts;
            const int yl = row >> 1, h = row & 1;
            bt[(yl * 2 + h) * kMS + part * 64 + lane] = cp[i];
        }
    };

    v16i rf[kMSub];
#pragma unroll
    for (int t = 0; t < kMSub; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) rf[t][v] = 0;
    v16i bias = {kBias, kBias, kBias, kBias, kBias, kBias, kBias, kBias,
                 kBias, kBias, kBias, kBias, kBias, kBias, kBias, kBias};
    asm volatile("" : "+v"(bias));   // kept in registers, not re-created per use
    // byte offset of lane (col, half)'s 16 operand bytes within a domain row pair
    const uint32_t lane_off = (uint32_t)(half * kMS + col) * 16u;
    const char *lds = reinterpret_cast<const char *>(s_lds);
    auto ldsb = [&](uint32_t off) { return *reinterpret_cast<const v4i *>(lds + off); };

    // A stage holds the tiles of a superblock's kSB blocks. While block h of
    // superblock sb is multiplied, block h of the next visited superblock is
    // loaded into registers and then written to the other stage; one barrier
    // per superblock makes both visible.
    int sb = next_sb(sblo);
    if (sb < sbhi) {
        const uint32_t w0 = ops_word(sb * kSB);
#pragma unroll
        for (int q = 0; q < kMaxUnits / 2; ++q) load_two(w0, 2 * q);
        for (int h = 0; h < kSB; ++h) {
            fetch(sb * kSB + h);
            store(0, h);
        }
    }
    __syncthreads();
    int cchunk = -1, stage = 0;
    while (sb < sbhi) {
        const int sbn = next_sb(sb + 1);
        const bool more = sbn < sbhi;
        for (int h = 0; h < kSB; ++h) {
            const int blk = sb * kSB + h;
            if (blk >= bhi) break;   // the last superblock of an odd block count
            if ((blk >> kTabShift) != cchunk) {
                // the operand loads (one block ahead) moved the lane tables to
                // this block's chunk
                cchunk = blk >> kTabShift;
                tdC = tdI;
                tbC = tbI;
            }
            const uint32_t desc = lane_word(tdC, blk), wb = lane_word(tbC, blk);
            // block h of the next superblock's domain tile (stored after this
            // block's products), and the operands of the next block multiplied,
            // loaded into the registers of each unit pair once it is done
            const int nxt = (h + 1 < kSB && blk + 1 < bhi) ? blk + 1 : (more ? sbn * kSB : blk);
            if (more) fetch(sbn * kSB + h);
            const uint32_t wn = ops_word(nxt);

            const int nu = (int)(wb >> 27);
            const int nc = (int)((desc >> 24) & 7u), nbe = 2 * nc + (int)((desc >> 27) & 15u);
            const uint32_t stage_off = (uint32_t)((stage * kSB + h) * kBTile) * 16u;
            // a leftover's word has a real flag for its own variable only
            const int lmask = (desc >> 31) ? kFlag1 : kFlag0;
#pragma unroll
            for (int q = 0; q < kMaxUnits / 2; ++q) {
                const int u0 = 2 * q, u1 = 2 * q + 1;
                const uint32_t o0 = stage_off + ((desc >> (3 * u0)) & 7u) * (2u * kMS * 16u) + lane_off;
                const uint32_t o1 = stage_off + ((desc >> (3 * u1)) & 7u) * (2u * kMS * 16u) + lane_off;
                if (u0 >= nu) {
                    // No unit. The words still pass through one VALU operation
                    // each: a path that left them where they are would make the
                    // compiler copy every path's results back (32 v_mov_b64 per
                    // pair of units).
                    int z = 0;
                    asm volatile("" : "+v"(z));
#pragma unroll
                    for (int t = 0; t < kMSub; ++t)
#pragma unroll
                        for (int v = 0; v < 16; ++v) rf[t][v] |= z;
                } else if (q < nc) {
                    // chained: a neighbour of only x0, then one of only x1
                    v16i e = mfma8(Aop[u1], ldsb(o1), mfma8(Aop[u0], ldsb(o0), bias));
#pragma unroll
                    for (int t = 0; t < kMSub; ++t) {
                        const v16i dd = e;
                        if (t + 1 < kMSub)
                            e = mfma8(Aop[u1], ldsb(o1 + (t + 1) * 512),
                                      mfma8(Aop[u0], ldsb(o0 + (t + 1) * 512), bias));
#pragma unroll
                        for (int v = 0; v < 16; ++v) rf[t][v] |= dd[v];
                    }
                } else if (u1 < nu) {
                    // two units: shared neighbours, or leftovers (from index nbe)
                    if (u1 < nbe) {
                        v16i e0 = mfma8(Aop[u0], ldsb(o0), bias);
                        v16i e1 = mfma8(Aop[u1], ldsb(o1), bias);
#pragma unroll
                        for (int t = 0; t < kMSub; ++t) {
                            v16i f0 = e0, f1 = e1;
                            if (t + 1 < kMSub) {
                                e0 = mfma8(Aop[u0], ldsb(o0 + (t + 1) * 512), bias);
                                e1 = mfma8(Aop[u1], ldsb(o1 + (t + 1) * 512), bias);
                            }
#pragma unroll
                            for (int v = 0; v < 16; ++v) rf[t][v] = rf[t][v] | f0[v] | f1[v];
                        }
                    } else {
                        const int m0 = u0 < nbe ? -1 : lmask;
                        v16i e0 = mfma8(Aop[u0], ldsb(o0), bias);
                        v16i e1 = mfma8(Aop[u1], ldsb(o1), bias);
#pragma unroll
                        for (int t = 0; t < kMSub; ++t) {
                            const v16i d0 = e0, d1 = e1;
                            if (t + 1 < kMSub) {
                                e0 = mfma8(Aop[u0], ldsb(o0 + (t + 1) * 512), bias);
                                e1 = mfma8(Aop[u1], ldsb(o1 + (t + 1) * 512), bias);
                            }
#pragma unroll
                            for (int v = 0; v < 16; ++v) {
                                // two v_and_or (the compiler would otherwise form
                                // two v_and and a v_or3: 5 % slower at step 1)
                                int r = (d0[v] & m0) | rf[t][v];
                                asm volatile("" : "+v"(r));
                                rf[t][v] = (d1[v] & lmask) | r;
                            }
                        }
                    }
                } else {
                    const int m0 = u0 < nbe ? -1 : lmask;
                    v16i e0 = mfma8(Aop[u0], ldsb(o0), bias);
#pragma unroll
                    for (int t = 0; t < kMSub; ++t) {
                        const v16i d0 = e0;
                        if (t + 1 < kMSub) e0 = mfma8(Aop[u0], ldsb(o0 + (t + 1) * 512), bias);
#pragma unroll
                        for (int v = 0; v < 16; ++v) rf[t][v] |= d0[v] & m0;   // one v_and_or each
                    }
                }
                load_two(wn, u0);   // this pair's registers now take the next block's operands
            }
            // The next superblock's tile goes to the stage every wave last read
            // in the previous superblock, before the barrier that ended it.
            if (more) store(stage ^ 1, h);
        }
        if (more) __syncthreads();
        stage ^= 1;
        sb = sbn;
    }

    if (nseg > 1) {
        // split step: OR this workgroup's unsupported values into A.kill
#pragma unroll
        for (int xi = 0; xi < kXW; ++xi) {
            if (!xvs[xi]) continue;
            const int flag = xi == 0 ? kFlag0 : kFlag1;
#pragma unroll
            for (int t = 0; t < kMSub; ++t) {
                const int slot = st0 + t * 32 + col;
                uint32_t m = 0;
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (rf[t][4 * g + r] & flag) m |= 1u << (8 * g + 4 * half + r);
                m |= (uint32_t)__shfl_xor((int)m, 32, 64);   // every lane executes it
                if (half == 0 && slot < nact && m)
                    atomicOr(A.kill + (int64_t)xs[xi] * A.capB + slot, m);
            }
        }
        return;
    }

    // epilogue: new domain bytes and per-state change / wipe-out masks
    int8_t *dnext = A.dom8[1];
#pragma unroll
    for (int xi = 0; xi < kXW; ++xi) {
        if (!xvs[xi]) continue;
        const int x = xs[xi];
        const int flag = xi == 0 ? kFlag0 : kFlag1;
#pragma unroll
        for (int t = 0; t < kMSub; ++t) {
            const int slot = st0 + t * 32 + col;
            const bool live = slot < nact;
            bool changed = false, nonempty = false;
            if (live) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    // rows a = 8g + 4*half + r, r = 0..3: bytes of half g/2 at 8(g%2) + 4*half
                    const int64_t off = dom_off(A, x, g >> 1, slot) + 8 * (g & 1) + 4 * half;
                    const uint32_t old = *reinterpret_cast<const uint32_t *>(din + off);
                    uint32_t keep = 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if ((rf[t][4 * g + r] & flag) == 0) keep |= 0xFFu << (8 * r);
                    const uint32_t nw = old & keep;
                    *reinterpret_cast<uint32_t *>(dnext + off) = nw;
                    changed |= nw != old;
                    nonempty |= nw != 0;
                }
            }
            // both lanes of a state column exchange their halves; the shuffles
            // run in every lane (no short-circuit), as ds_bpermute reads the
            // source lane's register
            const int other_changed = __shfl_xor((int)changed, 32, 64);
            const int other_nonempty = __shfl_xor((int)nonempty, 32, 64);
            changed = changed || other_changed != 0;
            nonempty = nonempty || other_nonempty != 0;
            const bool wiped = live && !nonempty;
            const uint64_t mc = __ballot(changed && live);
            const uint64_t mw = __ballot(wiped);
            if (lane == 0) {
                const int w = (st0 + t * 32) >> 5;
                A.chg[(int64_t)x * A.words + w] = (uint32_t)mc;
                A.wipe[(int64_t)x * A.words + w] = (uint32_t)mw;
            }
        }
    }
}

// After a split step: new domain bytes of every (x, active slot) from
// A.kill (which it clears), and the per-word change and wipe-out masks, as
// the unsplit kernel's epilogue writes them. Threads cover 64 slots of one
// variable per wave.
__global__ void mfma_split_finish_kernel(MArgs A, int k) {
    if (step_off(A, k) || A.ctl[2 + (k & 1)] <= 1) return;   // not a split step
    const int nact = A.cnt[(k - 1) & 1];
    const int64_t s64 = ((int64_t)nact + 63) / 64 * 64;
    const int64_t total = s64 * A.n;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool in = i < total;
        const int32_t x = in ? (int32_t)(i / s64) : 0;
        const int32_t slot = in ? (int32_t)(i - (int64_t)x * s64) : 0;
        const bool live = in && slot < nact;
        bool changed = false, nonempty = false;
        if (live) {
            uint32_t *kp = A.kill + (int64_t)x * A.capB + slot;
            const uint32_t m = *kp;
            if (m) *kp = 0;
            uint4 klo, khi;
            mask_to_bytes(~(uint64_t)m & 0xFFFFFFFFull, klo, khi);
            const uint4 lo = *reinterpret_cast<const uint4 *>(A.dom8[0] + dom_off(A, x, 0, slot));
            const uint4 hi = *reinterpret_cast<const uint4 *>(A.dom8[0] + dom_off(A, x, 1, slot));
            const uint4 nlo = make_uint4(lo.x & klo.x, lo.y & klo.y, lo.z & klo.z, lo.w & klo.w);
            const uint4 nhi = make_uint4(hi.x & khi.x, hi.y & khi.y, hi.z & khi.z, hi.w & khi.w);
            *reinterpret_cast<uint4 *>(A.dom8[1] + dom_off(A, x, 0, slot)) = nlo;
            *reinterpret_cast<uint4 *>(A.dom8[1] + dom_off(A, x, 1, slot)) = nhi;
            changed = m != 0 && ((nlo.x ^ lo.x) | (nlo.y ^ lo.y) | (nlo.z ^ lo.z) | (nlo.w ^ lo.w) |
                                 (nhi.x ^ hi.x) | (nhi.y ^ hi.y) | (nhi.z ^ hi.z) | (nhi.w ^ hi.w)) != 0;
            nonempty = (nlo.x | nlo.y | nlo.z | nlo.w | nhi.x | nhi.y | nhi.z | nhi.w) != 0;
        }
        const uint64_t mc = __ballot(changed);
        const uint64_t mw = __ballot(live && !nonempty);
        // a wave holds slots 64j .. 64j+63 of one variable: two mask words
        if (in && (lane & 31) == 0 && slot < nact) {
            const int w = slot >> 5;
            A.chg[(int64_t)x * A.words + w] = (uint32_t)(lane ? mc >> 32 : mc);
            A.wipe[(int64_t)x * A.words + w] = (uint32_t)(lane ? mw >> 32 : mw);
        }
    }
}

// Per slot word: OR of the change and wipe-out masks over all variables, and
// the sum of deg(x) over the variables that changed (support checks of the
// next step: every arc into a changed variable is re-examined).
// Block w (1024 threads): 32 groups of 32 lanes, lane b of a group summing
// for state bit b over the variables x = group, group + 32, ... (every lane
// of a group reads the same mask words, four variables' words in flight),
// then the groups' sums are added.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void mfma_reduce_kernel(MArgs A, int k) {
    constexpr int kGroups = kReduceThreads / 32;
    __shared__ uint32_t s_or[kGroups], s_wp[kGroups];
    __shared__ unsigned long long s_deg[kGroups][32];
    if (step_off(A, k)) return;
    const int nact = A.cnt[(k - 1) & 1];
    const int w = blockIdx.x;
    if (w * 32 >= nact) return;
    const int g = threadIdx.x >> 5, b = threadIdx.x & 31;
    uint32_t c_or = 0, w_or = 0;
    unsigned long long dsum = 0;
    for (int x0 = g; x0 < A.n; x0 += 4 * kGroups) {
        uint32_t c[4], wp[4];
        int32_t dg[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + i * kGroups;
            const bool in = x < A.n;
            c[i] = in ? A.chg[(int64_t)x * A.words + w] : 0u;
            wp[i] = in ? A.wipe[(int64_t)x * A.words + w] : 0u;
            dg[i] = in ? A.deg[x] : 0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c_or |= c[i];
            w_or |= wp[i];
            dsum += ((c[i] >> b) & 1u) ? (unsigned long long)dg[i] : 0ull;
        }
    }
    s_deg[g][b] = dsum;
    if (b == 0) {
        s_or[g] = c_or;
        s_wp[g] = w_or;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const int slot = w * 32 + threadIdx.x;
        if (slot < nact) {
            uint32_t o = 0, wp = 0;
            unsigned long long d = 0;
#pragma unroll
            for (int i = 0; i < kGroups; ++i) {
                o |= s_or[i];
                wp |= s_wp[i];
                d += s_deg[i][threadIdx.x];
            }
            MState &m = A.st[A.act[(k - 1) & 1][slot]];
            m.changed = (o >> threadIdx.x) & 1u;
            m.wiped |= (int32_t)((wp >> threadIdx.x) & 1u);
            m.degsum = d;
        }
    }
}

// Algorithm 1's loop test per state, the next step's active list, and the
// map from this step's slots to the next step's.
__global__ __launch_bounds__(1024) void mfma_finalize_kernel(MArgs A, int k) {
    __shared__ int32_t s_wave_tot[16];
    __shared__ int32_t s_base;
    if (step_off(A, k)) return;
    const int nact = A.cnt[(k - 1) & 1];
    const int32_t *act = A.act[(k - 1) & 1];
    int32_t *nxt = A.act[k & 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t maxs = A.max_sweeps > 0 ? A.max_sweeps : A.n * A.d + 1;
    __shared__ unsigned long long s_ops;
    if (threadIdx.x == 0) {
        s_base = 0;
        s_ops = 0;
    }
    // the next step's tile masks start empty (mfma_tile_changed_kernel fills them)
    for (int64_t i = threadIdx.x; i < (int64_t)A.words * 32 / kMS * A.nw32; i += blockDim.x) A.ych[i] = 0u;
    unsigned long long ops = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nact; c0 += 1024) {
        const int slot = c0 + threadIdx.x;
        bool keep = false;
        int32_t s = -1;
        if (slot < nact) {
            s = act[slot];
            MState &m = A.st[s];
            const bool changed = m.changed != 0;
            const bool stop_on_wipe = (A.mode == RAC_STOP_ON_WIPEOUT) && m.wiped;
            if (changed && !stop_on_wipe && k < maxs) {
                m.checks += (long long)m.degsum * A.d * A.d;
                ops += m.degsum;
                keep = true;
            } else {
                m.iters = k;
                m.status = m.wiped ? RAC_WIPEOUT : RAC_CONSISTENT;
                m.rc = (changed && !stop_on_wipe) ? RAC_ENOTCONVERGED : 0;
                m.done = 1;
            }
        }
        const uint64_t bal = __ballot(keep);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave_tot[wave] = __popcll(bal);
        __syncthreads();
        int off = s_base;
        for (int w = 0; w < wave; ++w) off += s_wave_tot[w];
        if (keep) {
            nxt[off + pre] = s;
            A.prev_slot[k & 1][off + pre] = slot;
        }
        if (slot < nact) A.slot_map[slot] = keep ? off + pre : -1;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += s_wave_tot[w];
            s_base += tot;
        }
        __syncthreads();
    }
    if (ops) atomicAdd(&s_ops, ops);
    __syncthreads();
    if (threadIdx.x == 0) {
        A.cnt[k & 1] = s_base;
        if (k + 1 <= kMaxTrackedSteps) A.stepops[k + 1] = s_ops;
        // Algorithm 1's loop, on the device: the matrix-core steps end when no
        // state goes on, or when the rest is few enough for the bit rows
        if (s_base == 0 || (A.handoff > 0 && s_base <= A.handoff)) {
            A.ctl[1] = k;
            A.ctl[0] = 1;
        } else {
            A.ctl[2 + ((k + 1) & 1)] = split_for(A, s_base);
        }
    }
}

// After the gather of step k: for each state tile of step k+1 (new slots) and
// variable y, whether y changed in step k in some state of the tile (bit y of
// the tile's words). A wave writes one word, 32 variables of one tile: lane l
// looks at the tile's new slots l, l + 64, ... through their old slots.
__global__ void mfma_tile_changed_kernel(MArgs A, int k) {
    if (step_off(A, k)) return;
    const int nnext = A.cnt[k & 1];
    const int64_t nwork = (int64_t)((nnext + kMS - 1) / kMS) * A.nw32;
    const int lane = threadIdx.x & 63, wpb = blockDim.x >> 6;
    const int32_t *prev = A.prev_slot[k & 1];
    for (int64_t wk = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); wk < nwork;
         wk += (int64_t)gridDim.x * wpb) {
        const int t = (int)(wk / A.nw32), wy = (int)(wk - (int64_t)t * A.nw32);
        int32_t old[kParts];
        bool ok[kParts];
#pragma unroll
        for (int h = 0; h < kParts; ++h) {
            const int j = t * kMS + h * 64 + lane;
            ok[h] = j < nnext;
            old[h] = ok[h] ? prev[j] : 0;
        }
        uint32_t word = 0;
        for (int yi = 0; yi < 32; ++yi) {
            const int y = wy * 32 + yi;
            if (y >= A.n) break;
            const uint32_t *row = A.chg + (int64_t)y * A.words;
            bool c = false;
#pragma unroll
            for (int h = 0; h < kParts; ++h)
                c |= ok[h] && ((row[old[h] >> 5] >> (old[h] & 31)) & 1u);
            if (__ballot(c)) word |= 1u << yi;
        }
        if (lane == 0) A.ych[(int64_t)t * A.nw32 + wy] = word;
    }
}

// After step k: the domains of the states that go on move to their new slots
// in the input buffer; the states that stopped write their final domains.
__global__ void mfma_gather_kernel(MArgs A, int k) {
    if (step_off(A, k)) return;
    const int nact = A.cnt[(k - 1) & 1];
    const int32_t *act = A.act[(k - 1) & 1];
    const int64_t total = (int64_t)nact * A.n;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < total; i += nth) {
        const int32_t x = (int32_t)(i / nact);
        const int32_t slot = (int32_t)(i - (int64_t)x * nact);
        const uint4 lo = *reinterpret_cast<const uint4 *>(A.dom8[1] + dom_off(A, x, 0, slot));
        const uint4 hi = *reinterpret_cast<const uint4 *>(A.dom8[1] + dom_off(A, x, 1, slot));
        const int32_t j = A.slot_map[slot];
        if (j >= 0) {
            *reinterpret_cast<uint4 *>(A.dom8[0] + dom_off(A, x, 0, j)) = lo;
            *reinterpret_cast<uint4 *>(A.dom8[0] + dom_off(A, x, 1, j)) = hi;
        } else {
            A.dout[(int64_t)act[slot] * A.n + x] = bytes_to_mask(lo, hi);
        }
    }
}

// Hand the P states still active after step k to the bit-row path: their
// domains D^(k) as masks, the variables step k changed (the @changed set the
// next step starts from, Proposition 2), and their state ids.
__global__ void mfma_handoff_kernel(MArgs A, int k, uint64_t *bits, uint8_t *changed,
                                    int32_t *ids) {
    const int P = A.cnt[k & 1];
    const int64_t total = (int64_t)P * A.n;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < total; i += nth) {
        const int64_t q = i / A.n;
        const int32_t x = (int32_t)(i - q * A.n);
        const int32_t s = A.act[k & 1][q];
        const int32_t slot = A.prev_slot[k & 1][q];
        const uint4 lo = *reinterpret_cast<const uint4 *>(A.dom8[0] + dom_off(A, x, 0, (int32_t)q));
        const uint4 hi = *reinterpret_cast<const uint4 *>(A.dom8[0] + dom_off(A, x, 1, (int32_t)q));
        bits[i] = bytes_to_mask(lo, hi);
        changed[i] = (uint8_t)((A.chg[(int64_t)x * A.words + (slot >> 5)] >> (slot & 31)) & 1u);
        if (x == 0) ids[q] = s;
    }
}

// Results of the bit-row path for the handed-off states: steps continue the
// count of the matrix-core steps, and the final domains go to the output.
__global__ void mfma_merge_kernel(MArgs A, int k, const uint64_t *bits, const int32_t *ids,
                                  const int32_t *it, const int32_t *stt, const long long *chk,
                                  const int32_t *brc) {
    const int P = A.cnt[k & 1];
    const int64_t total = (int64_t)P * A.n;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < total; i += nth) {
        const int64_t q = i / A.n;
        const int32_t x = (int32_t)(i - q * A.n);
        const int32_t s = ids[q];
        A.dout[(int64_t)s * A.n + x] = bits[i];
        if (x == 0) {
            MState &m = A.st[s];
            m.iters = k + it[q];
            m.status = stt[q];
            m.checks += chk[q];
            m.rc = (*brc & 1) ? RAC_ENOTCONVERGED : 0;
            m.done = 1;
        }
    }
}

// Per-state outputs (the domains were written as the states stopped).
__global__ void mfma_pack_kernel(MArgs A) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = tid; s < A.B; s += nth) {
        const MState &m = A.st[s];
        if (A.iters_out) A.iters_out[s] = m.iters;
        if (A.status_out) A.status_out[s] = m.status;
        if (A.checks_out) A.checks_out[s] = m.checks;
        if (A.rc_out && (m.rc != 0 || !m.done)) atomicOr(A.rc_out, m.done ? 1 : 4);
    }
}

// Row a of an arc as bits (bit b: (a,b) allowed); src = 2e + flip, the arc
// y->x of constraint e (flip = 1) holding column a of the constraint's rows.
__device__ __forceinline__ uint32_t arc_row32(const uint64_t *rel, int32_t src, int32_t d, int32_t a) {
    if (src < 0 || a >= d) return 0u;
    const uint64_t *R = rel + (int64_t)(src >> 1) * d;
    if ((src & 1) == 0) return (uint32_t)R[a];
    uint32_t row = 0;
    for (int b = 0; b < d; ++b) row |= (uint32_t)((R[b] >> a) & 1ull) << b;
    return row;
}

// Matrix-core A operands: operand o is R0 + 64 R1 as int8 bytes, R0 the
// relation of arc src[o].x (x0 -> y) and R1 that of arc src[o].y (x1 -> y),
// an absent arc (-1) contributing zeros; lane l holds row a = l % 32, values
// b = 16 (l / 32) .. +15, as the 32x32x32 int8 product reads its A operand.
__global__ void mfma_pack_ops_kernel(const uint64_t *rel, const int2 *src, int64_t nops, int32_t d,
                                     v4i *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (operand, lane)
    if (i >= nops * 64) return;
    const int64_t o = i >> 6;
    const int lane = (int)(i & 63), a = lane & 31, h = lane >> 5;
    const int2 sj = src[o];
    const uint32_t r0 = arc_row32(rel, sj.x, d, a) >> (16 * h);
    const uint32_t r1 = arc_row32(rel, sj.y, d, a) >> (16 * h);
    v4i w;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        w[q] = (int)(spread4((r0 >> (4 * q)) & 0xFu) | (spread4((r1 >> (4 * q)) & 0xFu) << 6));
    out[i] = w;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return set_error(e_ == hipErrorOutOfMemory ? RAC_ENOMEM : RAC_EHIP, "%s: %s", \
                             #call, hipGetErrorString(e_));                             \
    } while (0)

struct MfmaImpl {
    const int32_t *deg = nullptr;
    v4i *aop = nullptr;                          // matrix-core A operands
    uint32_t *udesc = nullptr, *ubase = nullptr; // per (pair, block) unit tables
    int64_t nops = 0;
    int32_t nblk = 0;
    int32_t capB = 0, words = 0;
    int8_t *dom8[2] = {nullptr, nullptr};
    uint32_t *chg = nullptr, *wipe = nullptr, *kill = nullptr, *ych = nullptr;
    unsigned long long *stepops = nullptr;
    int32_t *act[2] = {nullptr, nullptr};
    int32_t *prev_slot[2] = {nullptr, nullptr};
    int32_t *slot_map = nullptr;
    int32_t *ids = nullptr;
    int32_t *cnt = nullptr;
    MState *st = nullptr;
    uint64_t *hin = nullptr, *hout = nullptr;   // device staging for host calls
    int32_t *d_iters = nullptr, *d_status = nullptr, *d_rc = nullptr;
    long long *d_checks = nullptr;
    int32_t *h_cnt = nullptr;                    // pinned host copy of the control words and
                                                 // active counts, read once per round
    int32_t *ctl = nullptr;                      // device control words of the step loop
    struct Round {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Round> rounds;                   // captured rounds of steps, valid for graph_args
    MArgs graph_args{};
    bool graph_valid = false, graph_profiled = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_cnt = nullptr;
    hipEvent_t kev[2 * 64] = {};                 // step kernel timing (profiling)
    bool profiled = false;
    int32_t last_B = 0;
    int32_t last_k = 0;
    MArgs args{};
    int32_t *last_rc_ptr = nullptr;
};

static MfmaImpl *impl(MfmaData &md) { return reinterpret_cast<MfmaImpl *>(md.impl); }

template <typename T> static void mfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void mfma_release(MfmaData &md) {
    MfmaImpl *m = impl(md);
    if (!m) return;
    mfree(m->aop);
    mfree(m->udesc);
    mfree(m->ubase);
    mfree(m->dom8[0]);
    mfree(m->dom8[1]);
    mfree(m->chg);
    mfree(m->kill);
    mfree(m->wipe);
    mfree(m->ych);
    mfree(m->stepops);
    mfree(m->act[0]);
    mfree(m->act[1]);
    mfree(m->prev_slot[0]);
    mfree(m->prev_slot[1]);
    mfree(m->slot_map);
    mfree(m->ids);
    mfree(m->cnt);
    mfree(m->ctl);
    mfree(m->st);
    mfree(m->hin);
    mfree(m->hout);
    mfree(m->d_iters);
    mfree(m->d_status);
    mfree(m->d_rc);
    mfree(m->d_checks);
    if (m->h_cnt) (void)hipHostFree(m->h_cnt);
    for (auto &r : m->rounds) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
    }
    m->rounds.clear();
    if (m->ev0) (void)hipEventDestroy(m->ev0);
    if (m->ev1) (void)hipEventDestroy(m->ev1);
    if (m->ev_cnt) (void)hipEventDestroy(m->ev_cnt);
    for (auto &e : m->kev)
        if (e) (void)hipEventDestroy(e);
    delete m;
    md.impl = nullptr;
    md.ready = false;
}

bool mfma_auto_choice(int32_t d, int32_t n, int64_t arcs, int32_t B) {
    if (d > 32 || B < 64 || n < 8) return false;
    const double density = (double)arcs / ((double)n * (double)(n - 1));
    return density >= 0.25;
}

int mfma_ensure(MfmaData &md, int32_t n, int32_t d, int64_t arcs, const int32_t *row_ptr,
                const int32_t *nbr, const int32_t *deg, const uint64_t *rel,
                const int32_t *arc_src, const std::vector<int32_t> &h_row_ptr,
                hipStream_t stream) {
    if (md.ready) return RAC_OK;
    if (d > 32) return set_error(RAC_EUNSUPPORTED, "the matrix-core path needs d <= 32 (d=%d)", d);
    MfmaImpl *m = new MfmaImpl();
    md.impl = m;
    md.n = n;
    md.d = d;
    md.arcs = arcs;
    m->deg = deg;
    // neighbours of every variable, sorted, with their arcs (CSR order)
    std::vector<int32_t> h_nbr((size_t)arcs), h_src((size_t)arcs);
    if (arcs > 0) {
        HIP_OK(hipMemcpy(h_nbr.data(), nbr, (size_t)arcs * 4, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(h_src.data(), arc_src, (size_t)arcs * 4, hipMemcpyDeviceToHost));
    }
    std::vector<std::pair<int32_t, int32_t>> adj0, adj1;   // (y, arc source 2e + flip)
    auto nbrs = [&](int32_t x, std::vector<std::pair<int32_t, int32_t>> &out) {
        out.clear();
        if (x >= n) return;
        for (int32_t j = h_row_ptr[x]; j < h_row_ptr[x + 1]; ++j)
            out.push_back({h_nbr[(size_t)j], h_src[(size_t)j]});
        std::sort(out.begin(), out.end());
    };
    // per pair (x0 = 2p, x1 = 2p + 1) and block of 8 neighbours: the units
    // (chains of a neighbour of only x0 with one of only x1, then shared
    // neighbours, then leftovers), their operands and the unit tables
    const int32_t nblk = (n + kMY - 1) / kMY;
    const int32_t npairs = (n + 1) / 2;
    std::vector<uint32_t> udesc((size_t)npairs * nblk, 0), ubase((size_t)npairs * nblk, 0);
    std::vector<int2> ops;
    for (int32_t pr = 0; pr < npairs; ++pr) {
        nbrs(2 * pr, adj0);
        nbrs(2 * pr + 1, adj1);
        size_t i0 = 0, i1 = 0;
        for (int32_t b = 0; b < nblk; ++b) {
            const int32_t yend = (b + 1) * kMY;
            int32_t both[kMY][3], only0[kMY][2], only1[kMY][2];
            int nb = 0, n0 = 0, n1 = 0;
            while ((i0 < adj0.size() && adj0[i0].first < yend) || (i1 < adj1.size() && adj1[i1].first < yend)) {
                const int32_t y0 = i0 < adj0.size() ? adj0[i0].first : INT32_MAX;
                const int32_t y1 = i1 < adj1.size() ? adj1[i1].first : INT32_MAX;
                if (y0 == y1) {
                    both[nb][0] = y0 - b * kMY;
                    both[nb][1] = adj0[i0++].second;
                    both[nb++][2] = adj1[i1++].second;
                } else if (y0 < y1) {
                    only0[n0][0] = y0 - b * kMY;
                    only0[n0++][1] = adj0[i0++].second;
                } else {
                    only1[n1][0] = y1 - b * kMY;
                    only1[n1++][1] = adj1[i1++].second;
                }
            }
            const int nc = std::min(n0, n1);
            uint32_t desc = 0;
            int u = 0;
            const int64_t base = (int64_t)ops.size();
            for (int c = 0; c < nc; ++c) {
                desc |= (uint32_t)only0[c][0] << (3 * u++);
                ops.push_back(make_int2(only0[c][1], -1));
                desc |= (uint32_t)only1[c][0] << (3 * u++);
                ops.push_back(make_int2(-1, only1[c][1]));
            }
            for (int c = 0; c < nb; ++c) {
                desc |= (uint32_t)both[c][0] << (3 * u++);
                ops.push_back(make_int2(both[c][1], both[c][2]));
            }
            for (int c = nc; c < n0; ++c) {
                desc |= (uint32_t)only0[c][0] << (3 * u++);
                ops.push_back(make_int2(only0[c][1], -1));
            }
            for (int c = nc; c < n1; ++c) {
                desc |= (uint32_t)only1[c][0] << (3 * u++);
                ops.push_back(make_int2(-1, only1[c][1]));
            }
            desc |= (uint32_t)nc << 24 | (uint32_t)nb << 27 | (n1 > nc ? 1u << 31 : 0u);
            if (base > 0x7FFFFFF) return set_error(RAC_EUNSUPPORTED, "matrix-core operands exceed 2^27");
            udesc[(size_t)pr * nblk + b] = desc;
            ubase[(size_t)pr * nblk + b] = (uint32_t)base | (uint32_t)u << 27;
        }
    }
    m->nblk = nblk;
    m->nops = (int64_t)ops.size();
    HIP_OK(hipMalloc(&m->udesc, std::max<size_t>(1, udesc.size()) * 4));
    HIP_OK(hipMalloc(&m->ubase, std::max<size_t>(1, ubase.size()) * 4));
    HIP_OK(hipMemcpy(m->udesc, udesc.data(), udesc.size() * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(m->ubase, ubase.data(), ubase.size() * 4, hipMemcpyHostToDevice));
    // one spare operand past the end: a block with no units still loads its
    // (unused) first operand, which for the last blocks is operand nops
    HIP_OK(hipMalloc(&m->aop, (ops.size() + 1) * 1024));
    HIP_OK(hipMemset(m->aop, 0, (ops.size() + 1) * 1024));
    if (!ops.empty()) {
        int2 *d_ops = nullptr;
        HIP_OK(hipMalloc(&d_ops, ops.size() * sizeof(int2)));
        HIP_OK(hipMemcpy(d_ops, ops.data(), ops.size() * sizeof(int2), hipMemcpyHostToDevice));
        const int64_t threads = (int64_t)ops.size() * 64;
        hipLaunchKernelGGL(mfma_pack_ops_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                           stream, rel, d_ops, (int64_t)ops.size(), d, m->aop);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(stream));
        (void)hipFree(d_ops);
    }
    HIP_OK(hipFuncSetAttribute((const void *)mfma_sweep_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMSmem));
    HIP_OK(hipHostMalloc((void **)&m->h_cnt, sizeof(int32_t) * 8, hipHostMallocDefault));
    HIP_OK(hipMalloc(&m->ctl, sizeof(int32_t) * 4));
    HIP_OK(hipEventCreate(&m->ev0));
    HIP_OK(hipEventCreate(&m->ev1));
    HIP_OK(hipEventCreateWithFlags(&m->ev_cnt, hipEventDisableTiming));
    for (auto &e : m->kev) HIP_OK(hipEventCreate(&e));
    md.ready = true;
    return RAC_OK;
}

static int ensure_capacity(MfmaData &md, int32_t B) {
    MfmaImpl *m = impl(md);
    const int32_t capB = (B + kMS - 1) / kMS * kMS;
    if (capB <= m->capB) return RAC_OK;
    mfree(m->dom8[0]);
    mfree(m->dom8[1]);
    mfree(m->chg);
    mfree(m->kill);
    mfree(m->wipe);
    mfree(m->ych);
    mfree(m->stepops);
    mfree(m->act[0]);
    mfree(m->act[1]);
    mfree(m->prev_slot[0]);
    mfree(m->prev_slot[1]);
    mfree(m->slot_map);
    mfree(m->ids);
    mfree(m->cnt);
    mfree(m->st);
    mfree(m->hin);
    mfree(m->hout);
    mfree(m->d_iters);
    mfree(m->d_status);
    mfree(m->d_rc);
    mfree(m->d_checks);
    const size_t N32 = (size_t)md.n * 32;
    const int32_t words = capB / 32;
    HIP_OK(hipMalloc(&m->dom8[0], (size_t)capB * N32));
    HIP_OK(hipMalloc(&m->dom8[1], (size_t)capB * N32));
    HIP_OK(hipMalloc(&m->chg, (size_t)md.n * words * 4));
    HIP_OK(hipMalloc(&m->kill, (size_t)md.n * capB * 4));
    HIP_OK(hipMemset(m->kill, 0, (size_t)md.n * capB * 4));
    HIP_OK(hipMalloc(&m->wipe, (size_t)md.n * words * 4));
    HIP_OK(hipMalloc(&m->ych, (size_t)(capB / kMS) * ((md.n + 31) / 32) * 4));
    HIP_OK(hipMalloc(&m->stepops, (size_t)(kMaxTrackedSteps + 2) * 8));
    HIP_OK(hipMalloc(&m->act[0], (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->act[1], (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->prev_slot[0], (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->prev_slot[1], (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->slot_map, (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->ids, (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->cnt, 2 * 4));
    HIP_OK(hipMalloc(&m->st, (size_t)capB * sizeof(MState)));
    HIP_OK(hipMalloc(&m->hin, (size_t)capB * md.n * 8));
    HIP_OK(hipMalloc(&m->hout, (size_t)capB * md.n * 8));
    HIP_OK(hipMalloc(&m->d_iters, (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->d_status, (size_t)capB * 4));
    HIP_OK(hipMalloc(&m->d_rc, 4));
    HIP_OK(hipMalloc(&m->d_checks, (size_t)capB * 8));
    m->capB = capB;
    m->words = words;
    return RAC_OK;
}

static MArgs make_args(MfmaData &md, int32_t B, const uint64_t *din, uint64_t *dout,
                       int32_t *it, int32_t *stt, int32_t mode, int32_t max_sweeps) {
    MfmaImpl *m = impl(md);
    MArgs A;
    memset(&A, 0, sizeof(A));
    A.n = md.n;
    A.d = md.d;
    A.capB = m->capB;
    A.deg = m->deg;
    A.aop = m->aop;
    A.udesc = m->udesc;
    A.ubase = m->ubase;
    A.nblk = m->nblk;
    A.dom8[0] = m->dom8[0];
    A.dom8[1] = m->dom8[1];
    A.chg = m->chg;
    A.kill = m->kill;
    A.wipe = m->wipe;
    A.words = m->words;   // row stride of the mask matrices (capacity / 32)
    A.ych = m->ych;
    A.nw32 = (md.n + 31) / 32;
    A.stepops = m->stepops;
    A.ctl = m->ctl;
    A.ntiles_x = (md.n + kMX - 1) / kMX;
    {
        // RAC_MFMA_SEGMENTS forces the split of every step (tests)
        const char *e = getenv("RAC_MFMA_SEGMENTS");
        A.force_seg = e && *e ? std::max(0, std::min(atoi(e), kNsegMax)) : 0;
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            A.cus = cus;
        else
            A.cus = 256;
    }
    {
        const char *e = getenv("RAC_MFMA_SKIP");   // 0: every step re-examines every arc
        A.skip = (e && *e) ? (atoi(e) != 0) : 1;
    }
    A.act[0] = m->act[0];
    A.act[1] = m->act[1];
    A.prev_slot[0] = m->prev_slot[0];
    A.prev_slot[1] = m->prev_slot[1];
    A.slot_map = m->slot_map;
    A.cnt = m->cnt;
    A.st = m->st;
    A.mode = mode;
    A.max_sweeps = max_sweeps;
    A.B = B;
    A.xcd_map = 1;
    A.checks1 = md.arcs * md.d * md.d;
    A.din = din;
    A.dout = dout;
    A.iters_out = it;
    A.status_out = stt;
    A.rc_out = m->d_rc;   // the pack kernel also ORs the per-state codes into it
    A.checks_out = m->d_checks;
    return A;
}

#define RC_OK(expr)                    \
    do {                               \
        const int rc_ = (expr);        \
        if (rc_ != RAC_OK) return rc_; \
    } while (0)

// Kernel node of a round graph, chained after *prev.
static int round_node(hipGraph_t g, hipGraphNode_t *prev, const void *func, dim3 grid, dim3 block,
                      size_t smem, void **params) {
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(func);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)smem;
    kp.kernelParams = params;
    hipGraphNode_t node;
    HIP_OK(hipGraphAddKernelNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, &kp));
    *prev = node;
    return RAC_OK;
}

// Event record node of a round graph (per-launch timing), chained after *prev.
static int round_event(hipGraph_t g, hipGraphNode_t *prev, hipEvent_t ev) {
    hipGraphNode_t node;
    HIP_OK(hipGraphAddEventRecordNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, ev));
    *prev = node;
    return RAC_OK;
}

// Steps per round: 4, 4, 8, 16, 32, then 64.
static int mfma_round_steps(int r) { return r < 2 ? 4 : (r >= 5 ? 64 : 4 << (r - 1)); }

// Enqueues init and rounds of matrix-core steps. Whether the steps go on,
// how many workgroups a step splits into, and when the few states left move
// to the bit rows are decided on the device (finalise kernel); the host reads
// the control words once per round, and replays a captured graph per round
// when the arguments are those of the last call.
static int run_steps(MfmaData &md, const MArgs &A, bool profile, hipStream_t stream,
                     int32_t *k_out, int32_t *p_out) {
    MfmaImpl *m = impl(md);
    m->profiled = profile;
    m->args = A;
    const int ntiles_s = (A.words * 32 + kMS - 1) / kMS;
    // one workgroup per (x-tile, state tile) of the whole batch, times a
    // forced split count (tests); a split step uses the idle tiles' workgroups
    const int fgrid = A.force_seg > 0 ? A.force_seg : 1;
    const int sweep_blocks = ((A.ntiles_x + 7) / 8) * 8 * ntiles_s * fgrid;
    const int init_blocks = (int)std::min<int64_t>(4096, ((int64_t)A.B * A.n + 255) / 256);
    const int64_t thr64 = ((int64_t)A.B + 63) / 64 * 64 * A.n;
    const unsigned small_blocks = (unsigned)std::min<int64_t>(4096, (thr64 + 255) / 256);
    // a split step's finish kernel strides over its states (no step of the
    // batch's first rounds splits, and an idle grid still costs its launch);
    // the tile-change kernel has one wave per word of a state tile
    const unsigned split_blocks = std::min<unsigned>(small_blocks, 1024u);
    const unsigned tc_blocks = (unsigned)std::max<int64_t>(
        1, (((int64_t)A.B + kMS - 1) / kMS * A.nw32 + 3) / 4);
    const int32_t maxs = A.max_sweeps > 0 ? A.max_sweeps : A.n * A.d + 1;
    // rounds are replayed graphs, also when profiling: the timing events are
    // nodes of the graphs (RAC_MFMA_GRAPHS=0: direct launches)
    const char *eg = getenv("RAC_MFMA_GRAPHS");
    const bool graphs = !(eg && *eg && atoi(eg) == 0);
    if (graphs && !(m->graph_valid && m->graph_profiled == profile &&
                    memcmp(&m->graph_args, &A, sizeof(MArgs)) == 0)) {
        for (auto &r : m->rounds) {
            if (r.exec) (void)hipGraphExecDestroy(r.exec);
            if (r.graph) (void)hipGraphDestroy(r.graph);
        }
        m->rounds.clear();
        m->graph_args = A;
        m->graph_valid = true;
        m->graph_profiled = profile;
    }
    HIP_OK(hipEventRecord(m->ev0, stream));
    hipLaunchKernelGGL(mfma_init_kernel, dim3(init_blocks), dim3(256), 0, stream, A);
    int k = 0;
    for (int r = 0; k < maxs; ++r) {
        const int K = std::min(mfma_round_steps(r), maxs - k);
        if (graphs) {
            if ((int)m->rounds.size() <= r) m->rounds.resize((size_t)r + 1);
            MfmaImpl::Round &rd = m->rounds[(size_t)r];
            if (!rd.exec) {
                HIP_OK(hipGraphCreate(&rd.graph, 0));
                MArgs args = A;
                int nsm = fgrid;
                std::vector<int> ks((size_t)K);
                hipGraphNode_t prev = nullptr;
                for (int i = 0; i < K; ++i) {
                    ks[(size_t)i] = k + 1 + i;
                    void *p2[2] = {&args, &ks[(size_t)i]};
                    void *p3[3] = {&args, &ks[(size_t)i], &nsm};
                    const int kk = ks[(size_t)i];
                    const bool timed = profile && kk <= 64;
                    if (timed) RC_OK(round_event(rd.graph, &prev, m->kev[2 * (kk - 1)]));
                    RC_OK(round_node(rd.graph, &prev, (const void *)mfma_sweep_kernel, dim3(sweep_blocks),
                                       dim3(kMThreads), kMSmem, p3));
                    RC_OK(round_node(rd.graph, &prev, (const void *)mfma_split_finish_kernel,
                                       dim3(split_blocks), dim3(256), 0, p2));
                    if (timed) RC_OK(round_event(rd.graph, &prev, m->kev[2 * (kk - 1) + 1]));
                    RC_OK(round_node(rd.graph, &prev, (const void *)mfma_reduce_kernel,
                                       dim3((A.B + 31) / 32), dim3(kReduceThreads), 0, p2));
                    RC_OK(round_node(rd.graph, &prev, (const void *)mfma_finalize_kernel, dim3(1),
                                       dim3(1024), 0, p2));
                    RC_OK(round_node(rd.graph, &prev, (const void *)mfma_gather_kernel, dim3(init_blocks),
                                       dim3(256), 0, p2));
                    if (A.skip)
                        RC_OK(round_node(rd.graph, &prev, (const void *)mfma_tile_changed_kernel,
                                           dim3(tc_blocks), dim3(256), 0, p2));
                }
                HIP_OK(hipGraphInstantiate(&rd.exec, rd.graph, nullptr, nullptr, 0));
            }
            HIP_OK(hipGraphLaunch(rd.exec, stream));
            k += K;
        } else {
            for (int i = 0; i < K; ++i) {
                ++k;
                const bool timed = profile && k <= 64;
                if (timed) HIP_OK(hipEventRecord(m->kev[2 * (k - 1)], stream));
                hipLaunchKernelGGL(mfma_sweep_kernel, dim3(sweep_blocks), dim3(kMThreads), kMSmem, stream,
                                   A, k, fgrid);
                hipLaunchKernelGGL(mfma_split_finish_kernel, dim3(split_blocks), dim3(256), 0, stream, A, k);
                if (timed) HIP_OK(hipEventRecord(m->kev[2 * (k - 1) + 1], stream));
                hipLaunchKernelGGL(mfma_reduce_kernel, dim3((A.B + 31) / 32), dim3(kReduceThreads), 0, stream, A, k);
                hipLaunchKernelGGL(mfma_finalize_kernel, dim3(1), dim3(1024), 0, stream, A, k);
                hipLaunchKernelGGL(mfma_gather_kernel, dim3(init_blocks), dim3(256), 0, stream, A, k);
                if (A.skip)
                    hipLaunchKernelGGL(mfma_tile_changed_kernel, dim3(tc_blocks), dim3(256), 0, stream,
                                       A, k);
            }
        }
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(m->h_cnt, A.ctl, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipMemcpyAsync(m->h_cnt + 4, A.cnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipEventRecord(m->ev_cnt, stream));
        HIP_OK(hipEventSynchronize(m->ev_cnt));
        if (m->h_cnt[0]) break;
    }
    // the steps ended at step kd: no state went on (left = 0), or `left`
    // states remain for the bit rows; at the step cap every state stopped
    const int32_t kd = m->h_cnt[0] ? m->h_cnt[1] : k;
    const int32_t left = m->h_cnt[0] ? m->h_cnt[4 + (kd & 1)] : 0;
    m->last_k = kd;
    *k_out = kd;
    *p_out = left;
    return RAC_OK;
}

int mfma_start(MfmaData &md, int32_t B, const uint64_t *d_in, uint64_t *d_out, int32_t mode,
               int32_t max_sweeps, int32_t profile, int32_t handoff, hipStream_t stream,
               int32_t *k_out, int32_t *p_out) {
    int rc = ensure_capacity(md, B);
    if (rc) return rc;
    MfmaImpl *m = impl(md);
    MArgs A = make_args(md, B, d_in, d_out, nullptr, nullptr, mode, max_sweeps);
    m->last_B = B;
    A.handoff = handoff;
    return run_steps(md, A, profile != 0, stream, k_out, p_out);
}

int mfma_handoff(MfmaData &md, int32_t k, uint64_t *d_bits, uint8_t *d_changed, hipStream_t stream) {
    MfmaImpl *m = impl(md);
    const MArgs &A = m->args;
    const int blocks = (int)std::min<int64_t>(4096, ((int64_t)A.B * A.n + 255) / 256);
    hipLaunchKernelGGL(mfma_handoff_kernel, dim3(blocks), dim3(256), 0, stream, A, k, d_bits,
                       d_changed, m->ids);
    HIP_OK(hipGetLastError());
    return RAC_OK;
}

int mfma_merge(MfmaData &md, int32_t k, const uint64_t *d_bits, const int32_t *d_it,
               const int32_t *d_st, const long long *d_chk, const int32_t *d_rc,
               hipStream_t stream) {
    MfmaImpl *m = impl(md);
    const MArgs &A = m->args;
    const int blocks = (int)std::min<int64_t>(4096, ((int64_t)A.B * A.n + 255) / 256);
    hipLaunchKernelGGL(mfma_merge_kernel, dim3(blocks), dim3(256), 0, stream, A, k, d_bits, m->ids,
                       d_it, d_st, d_chk, d_rc);
    HIP_OK(hipGetLastError());
    return RAC_OK;
}

int mfma_finish(MfmaData &md, int32_t *d_iters, int32_t *d_status, hipStream_t stream) {
    MfmaImpl *m = impl(md);
    MArgs A = m->args;
    A.iters_out = d_iters;
    A.status_out = d_status;
    const int blocks = (int)std::min<int64_t>(4096, ((int64_t)A.B + 255) / 256);
    hipLaunchKernelGGL(mfma_pack_kernel, dim3(blocks), dim3(256), 0, stream, A);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(m->ev1, stream));
    return RAC_OK;
}

static int rc_of(int32_t v) {
    if (v & 4) return set_error(RAC_ETIMEOUT, "matrix-core path: a state did not finish");
    if (v & 1) return set_error(RAC_ENOTCONVERGED, "max_sweeps reached before the fixpoint");
    return RAC_OK;
}

static void collect_stats(MfmaData &md, int32_t B, const std::vector<long long> &checks,
                          const std::vector<int32_t> &iters,
                          const std::vector<unsigned long long> &stepops, rac_stats *stats) {
    MfmaImpl *m = impl(md);
    memset(stats, 0, sizeof(*stats));
    int32_t max_it = 0;
    for (int32_t s = 0; s < B; ++s) {
        stats->support_checks += checks[(size_t)s];
        stats->sweeps += iters[(size_t)s];
        max_it = std::max(max_it, iters[(size_t)s]);
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, m->ev0, m->ev1);
    stats->device_ms = ms;
    stats->path = RAC_PATH_MFMA;
    stats->relation_bytes = m->nops * 1024;   // the matrix-core operands, read once per state tile
    // the matrix-core steps' work on the arcs they re-examine (Proposition 2):
    // step 1 every arc of every state, step k >= 2 the arcs into the
    // variables each active state changed in step k-1
    long long arcs_examined = md.arcs * (long long)B;
    const int32_t kt = std::min(m->last_k, kMaxTrackedSteps);
    for (int32_t k = 2; k <= kt; ++k) arcs_examined += (long long)stepops[(size_t)k];
    stats->algo_ops = 2ll * md.d * md.d * arcs_examined;
    if (m->profiled) {
        // the step kernels that had work: steps 1..min(max iters, last step)
        const int32_t kl = std::min(std::min(max_it, m->last_k), 64);
        for (int32_t k = 1; k <= kl; ++k) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, m->kev[2 * (k - 1)], m->kev[2 * (k - 1) + 1]);
            if (k == 1) stats->first_kernel_ms = t;
            stats->kernel_ms += t;
        }
        stats->kernel_launches = kl;
    }
}

int mfma_collect(MfmaData &md, rac_stats *stats) {
    MfmaImpl *m = impl(md);
    const int32_t B = m->last_B;
    HIP_OK(hipEventSynchronize(m->ev1));
    std::vector<MState> hs((size_t)B);
    int32_t hrc = 0;
    HIP_OK(hipMemcpy(hs.data(), m->st, (size_t)B * sizeof(MState), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&hrc, m->d_rc, 4, hipMemcpyDeviceToHost));
    std::vector<long long> hc((size_t)B);
    std::vector<int32_t> hi((size_t)B);
    for (int32_t s = 0; s < B; ++s) {
        hc[(size_t)s] = hs[(size_t)s].checks;
        hi[(size_t)s] = hs[(size_t)s].iters;
    }
    std::vector<unsigned long long> ops((size_t)kMaxTrackedSteps + 2, 0);
    HIP_OK(hipMemcpy(ops.data(), m->stepops, ops.size() * 8, hipMemcpyDeviceToHost));
    collect_stats(md, B, hc, hi, ops, stats);
    return rc_of(hrc);
}

}  // namespace rac
