// Internal declarations of the MI355X multipole gravity library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpg.h"
#include "batch_order.h"
#include "ksplit.h"

namespace mpg {

typedef __bf16 bf16;

// A store, non-temporal with NT (streamed past the caches: the fused batch
// kernel's stage outputs, so that its per-item L2 write-backs find few
// dirty lines).
template <bool NT, typename V>
__device__ __forceinline__ void store(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Thread-local error text behind mpg_last_error().
void set_error(const std::string &msg);

// Tile constants shared by the plan layout and the kernels.
constexpr int kSplitTile = 128;  // split-BF16 GEMM tiles are kSplitTile x kSplitTile
constexpr int kF64Tile1 = 128;   // FP64 GEMM1 tiles are kF64Tile1 x kF64Tile1
constexpr int kF64Tile2 = 64;    // FP64 GEMM2 tiles are kF64Tile2 x kF64Tile2
constexpr int kColPad = 32;    // each m-parity column block is padded to this
constexpr int kColSlack = 128; // zero rows after the last column block
constexpr int kAngPad = 128;   // angular dimension padded to this

// Split-BF16 operands (rho+-, U, M, Q) are stored as tile-slab blocks: an
// operand with tiles of kSplitTile rows and K slabs of kSlabK holds, for
// each (tile, slab), the three bf16 pieces (h, m, l) of that 128x32
// submatrix one after the other, block after block in slab order:
//   element (tile, slab, piece, r, k) at ((tile*slabs + slab)*3 + piece)*kBlk + blk_pos(r, k).
// Inside a piece the 16-byte chunk (r, k/8) sits at 4r + ((k/8) ^ ((r/4)%4)):
// a block is copied to LDS as is, and the GEMMs' fragment reads of 16
// consecutive rows at one k chunk then fall into distinct LDS banks.
constexpr int kSlabK = 32;
constexpr int kBlk = kSplitTile * kSlabK;
__host__ __device__ inline int blk_pos(int r, int k) { return (4 * r + ((k >> 3) ^ ((r >> 2) & 3))) * 8 + (k & 7); }

// Column units of GEMM1 blocks (nb = 2: pairs of kSplitTile-column tiles;
// nb = 1: single tiles) among the `units` units of a parity block, whose
// leading six_cols columns take six products: the units holding any of them.
__host__ __device__ inline int six_units(int six_cols, int units, int nb) {
    const int n = (six_cols + nb * kSplitTile - 1) / (nb * kSplitTile);
    return n < units ? n : units;
}

// Leading three-product slabs of a K walk of nsl slabs that runs from the
// top of a column block down, whose lowest six_sl slabs take six products:
// rounded down to an even count (so one more slab may take six).
__host__ __device__ inline int three_slabs(int nsl, int six_sl) {
    const int n3 = nsl - six_sl > 0 ? nsl - six_sl : 0;
    return n3 == nsl ? n3 : (n3 & ~1);
}

// Table layout of a plan (all device arrays are owned by the plan).
//
// Columns are the real moment indices permuted so that even-m columns come
// first (block E, padded to ne_p) and odd-m columns second (block O, padded
// to no_p); np = ne_p + no_p.  Without the Yin/Yang fold there is a single
// block holding every column (no_p = 0).
struct Plan {
    // grid
    int n_patches = 0, n_r = 0, n_theta = 0, n_phi = 0, n_ang = 0;
    double theta0 = 0, phi0 = 0, dtheta = 0, dphi = 0;
    int lmax = 0, n_lm = 0, precision = MPG_FP64, max_fields = 1;
    bool split() const { return precision != MPG_FP64; }
    // overlap geometry of a symmetric Yin-Yang pair (used when no w is given)
    double ovl_sc = 0, ovl_kap = 0;
    int ovl_kap_inf = 0;
    bool fold = false;
    double G = 1.0;
    bool eval_centre = false;  // Phi at the cells' angular centres instead of their upper vertices
    hipStream_t stream = nullptr;
    int device = 0;

    // column layout
    int n_e = 0, n_o = 0, ne_p = 0, no_p = 0, np = 0, np_alloc = 0;
    int n_angp = 0;            // n_ang padded to kAngPad
    // split forms: leading columns of the even / odd block (multiples of
    // kSlabK) whose products take all six bf16 piece products; the other
    // columns take three (all columns for MPG_SPLIT_BF16)
    int six_e = 0, six_o = 0;
    // patch blocks of the contractions: 1 under the fold (and for one
    // patch), n_patches on the general path, whose GEMM1 K and GEMM2 N run
    // over the cells of every patch, patch after patch (kang = npat*n_angp)
    int npat = 1;
    int kang() const { return npat * n_angp; }
    // per-patch method (the comparison method of Sec. 4.3): the moments of
    // every patch in its own frame (GEMM1 and the scans see n_patches
    // single-patch fields per field), and an expansion whose K runs over
    // the moment sets of every patch (kq = n_patches*np) and whose N runs
    // over the cells of every patch
    bool per_patch = false;
    int nq() const { return per_patch ? n_patches : 1; }
    int kq() const { return nq() * np; }
    int n2() const { return per_patch ? n_patches * n_angp : kang(); }
    // single-patch fields that GEMM1 and the scans see for n_fields fields
    int vfields(int n_fields) const { return per_patch ? n_fields * n_patches : n_fields; }

    // separable method: in each patch's own frame the cell weights factor
    // over (theta, phi), so each contraction runs as a phi transform of
    // every (field, patch, shell, theta row) row, a theta contraction per
    // order u, and a rotation to or from the common frame per degree.  Phi
    // columns c: 0 is the order-0 column (constant factors: summed outside
    // the MFMA tiles), then C of u = 1..lmax and S of u = 1..lmax, each
    // padded to 16.  On a phi grid symmetric about 0 with an even cell
    // count (sep_mir) cells k and n_phi-1-k are taken together: the C
    // columns see their sum, the S columns their difference.
    bool sep = false, sep_mir = false;
    int sep_ce = 0, sep_co = 0;  // C / S phi columns of orders >= 1 (multiples of 16)
    int sep_lp = 0;              // degree slots per phi column (lmax + 1 rounded up to 16)
    int sep_kh = 0, sep_khp = 0; // cells of a row the moments' transform walks (n_phi/2 mirrored), padded to 16
    int sep_kx = 0;              // evaluation points of a row the expansion's transform computes
    int *sep_m = nullptr;        // [nc] order u of a phi column, -1 = pad
    int *sep_coff = nullptr;     // [nc] first slot of a phi column (slots of degrees u..lmax)
    int *sep_cslot = nullptr;    // [n_lm] slot of a real index
    int2 *sep_kxy = nullptr;     // [sep_kx] cell of an evaluation point and its mirror cell (-1: none)
    long long *sep_xoff = nullptr;  // [lmax + 2] offsets of the degrees' rotations
    int *sep_perm = nullptr;     // [n_lm] column of a real index
    double *sep_f1 = nullptr;    // [sep_khp][nc] moments' phi factors (C_k^u, S_k^u)
    double *sep_t1 = nullptr;    // [nc][sep_lp][n_theta] moments' theta factors (s_lu T_j^{lu})
    double *sep_t2 = nullptr;    // [nc][sep_lp][n_theta] expansion's theta factors (-G s_lu P_l^u)
    double *sep_f2 = nullptr;    // [nc][sep_kx] expansion's phi factors
    double *sep_x1 = nullptr;    // rotations local -> common frame (moments)
    double *sep_x2 = nullptr;    // rotations common frame -> local (expansion)
    // split forms of the separable method: the phi transforms in six bf16
    // piece products with FP32 accumulation (tiles of 32 columns: C rows
    // [0, 32 sep_nt2), S rows after them)
    int sep_nt2 = 0;             // 32-column tiles per block (C or S) of the moments' transform
    int sep_kxp = 0;             // sep_kx rounded up to 64
    bf16 *sep_f1s = nullptr;     // [3][64 sep_nt2][sep_khp] pieces of the moments' phi factors
    bf16 *sep_f2s = nullptr;     // [3][sep_kxp][2 sep_ce] pieces of the expansion's phi factors (columns 1..)
    double *sep_A = nullptr;     // [n_lm][sep_ldv()] local moments / local expansion coefficients (by slot)
    double *sep_F = nullptr;     // [nc][n_theta][sep_ldv()] phi transforms (moments, then expansion)
    int sep_nc() const { return 1 + sep_ce + sep_co; }
    // (field, patch, shell) rows v, and their count padded to 128
    int sep_vrows() const { return max_fields * n_patches * n_r; }
    int sep_ldv() const { return (sep_vrows() + 127) / 128 * 128; }

    int *col_src = nullptr;    // [np_alloc] real index of a permuted column, -1 = pad
    int *col_l = nullptr;      // [np_alloc] degree, -1 = pad
    double *Ut = nullptr;      // [np_alloc][kang]  U of the npat patch blocks, K(angular)-contiguous
    double *Qt = nullptr;      // [n2][kq]          Q of the npat patch blocks (per patch: Q of patch p's
                               //                   cells in patch g's frame at [p][jk][g][q]), K(lm)-contiguous
    double *coef = nullptr;    // [n_r][lmax+1][4] radial recurrence coefficients
    double *w = nullptr;       // [npat][n_ang] overlap weights
    bf16 *Us = nullptr;        // split U: tiles = GEMM1 column tiles, slabs = kang/32 (tile-slab blocks)
    bf16 *Qs = nullptr;        // split Q: tiles = n2/128 angular tiles, slabs = kq/32

    // work space (sized for max_fields)
    int splitk = 1;            // K splits of the moment contraction (work space holds this many)
    int splitk_sel = 0;        // chosen by mpg_autotune (0: heuristic)
    int scan_chunks = 16;      // shell chunks per column in the radial scan
    int gemm1_rows = 1;        // moment blocks, split forms: 1 = 128 rows x 256 columns, 2 = 256 x 128;
                               // FP64: 1 = 128 x 128 tiles, 2 = 64 x 64
    int gemm1_rows_batch = 1;  // the same choice for batched solves
    int gemm2_rows = 1;        // split expansion blocks: 1 = 128 rows x 256 cells, 2 = 256 x 128
    int tune_epoch = 0;        // raised whenever the choices above change (batched solves rebuild)
    double *Bpart = nullptr;   // [splitk][rows][np]
    double *Bred = nullptr;    // [rows][np]
    double *M = nullptr;       // [rows][np]
    bf16 *Ms = nullptr;        // split M: tiles = row tiles of (field, shell), slabs = kq/32
    bf16 *A_split = nullptr;   // split input rho (+-): [fold ? 2 : 1] planes of row tiles x kang/32 slabs

    // rows of GEMM1 and the scans (per patch: n_patches per field and shell)
    int rows_alloc() const { return vfields(max_fields) * n_r; }
    int row_tiles() const { return (rows_alloc() + kSplitTile - 1) / kSplitTile; }
    // row tiles of the expansion's (field, shell) rows
    int out_row_tiles() const { return (max_fields * n_r + kSplitTile - 1) / kSplitTile; }
    // GEMM1 column tiles: even-m block tiles, then odd-m block tiles
    int tiles_e() const { return fold ? (ne_p + kSplitTile - 1) / kSplitTile : (np + kSplitTile - 1) / kSplitTile; }
    int tiles_o() const { return fold ? (no_p + kSplitTile - 1) / kSplitTile : 0; }

    // optional stage timing (events recorded on the plan's stream)
    bool timing = false;
    std::vector<hipEvent_t> *events[4] = {nullptr, nullptr, nullptr, nullptr};  // start/stop pairs
};

// ---- batch work descriptions ---------------------------------------------

// One work item of a persistent batch kernel: field f and tile coordinates.
struct BatchItem {
    int f, a, b, c;
};

// Per-field completion tracking of a batched solve: when a block of an
// expansion kernel has finished an item of field f (every wave past the
// item-queue barrier), its first thread raises stamps[f] to the device
// wall clock, so stamps[f] ends as the time the field's last item was done.
// stamps[n] is the batch's start; stamps[n + 1] takes the stamp of "no
// item yet" (the first fetch of a block).
struct BatchTrack {
    unsigned long long *stamps;  // [n + 2]
    int n;
};

// Item queue of the persistent batch kernels: a block's next item index
// (all threads get the same), after stamping the previous item's field
// (prev_f, or -1 before the first).  The stamp and the fetch share one
// first-thread section, so the loop around it keeps a single structure.
__device__ __forceinline__ int next_item_tracked(int *head, int *slot, const BatchTrack &t, int prev_f) {
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(t.stamps + (prev_f >= 0 ? prev_f : t.n + 1), (unsigned long long)wall_clock64());
        *slot = atomicAdd(head, 1);
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

// Control block of the fused batch kernel (device pointers): the queue
// head, per field and stage the items finished and the items in all
// ([n][kFusedStages] each), a status word that a wait sets to 1 when it
// gives up (the kernel then drains; the host reads it back), and the
// per-field completion stamps ([n + 2]: stamps[n] is the start).  A wait
// for a stage gives up after spin_limit polls (about 0.25 us each).
struct FusedCtl {
    int *head, *done;
    const int *need;
    int *status;
    unsigned long long *stamps;
    int n, spin_limit;
};

// Arguments of one field's split-BF16 contractions.
struct SplitArgs {
    const void *rho;
    void *phi;
    int io_f64;
    int rows, n_r, n_ang, n_angp, np, ne_p, fold;
    int n_patches, kang;  // patches of a field; npat*n_angp (GEMM1 K, GEMM2 N)
    int nq, kq;           // GEMM2 K: moment sets (per-patch method) and their total length
    int tiles_e, tiles_o;  // GEMM1 column tiles of the even / odd block
    int kchunk, splitk;    // GEMM1 K per split, number of splits
    const bf16 *U, *Q, *M;  // split tables and moments (tile-slab blocks)
    double *Bpart;
    bf16 *A;                // split input (tile-slab blocks, one plane per parity)
    int row_tiles;          // row tiles of a plane of A (and of M)
    int ks1, ks2;           // slabs of GEMM1 (kang/32) and GEMM2 (np/32)
    int six_e, six_o;       // leading columns of each block with six products (see Plan)
    int g1_rows, g2_rows;   // block shapes: 1 = 128 rows x 256 columns, 2 = 256 x 128 (see Plan)
};

// Arguments of one field's FP64 contractions.
struct F64Args {
    const void *rho;
    void *phi;
    int io_f64;
    int rows, n_r, n_ang, n_angp, np, ne_p, fold;
    int n_patches, kang;  // patches of a field; npat*n_angp (GEMM1 K, GEMM2 N)
    int nq, kq;           // GEMM2 K: moment sets (per-patch method) and their total length
    int tiles_e, tiles_o;  // GEMM1 column tiles of the even / odd block
    int t1;                // GEMM1 tile side (128, or 64: the plan's second moment shape)
    int kchunk, splitk;
    const double *Ut, *Qt, *M;
    double *Bpart;
};

// Arguments of one field's radial scans.
struct ScanArgs {
    const double *Bpart;
    int splitk, n_fields, n_r, np, L;
    const int *col_l;
    const double *coef;
    double *Bred, *M;
    bf16 *Ms;        // split copy of M (tile-slab blocks), or null
    int ks2;         // its slabs per row tile (kq/32)
    int pp;          // per-patch method: single-patch fields per field (its row (f, shell), column
                     // (patch, q) in Ms), else 0
    int col_blocks;  // blocks of 64 columns
    int chunks;      // shell chunks per column (1..16, at most n_r)
};

// ---- kernels launchers (each returns hipError_t of the launch) ----------

// table build (tables.hip)
// host_w: NULL, or n_ang weights shared by every patch block, or
// (w_per_patch) npat*n_ang
hipError_t build_tables(Plan &p, const double *host_euler, const double *host_r_edges,
                        const double *host_w, int w_per_patch);

// copy the FP64 tables out in the real index (tables.hip)
hipError_t export_tables(const Plan &p, double *U, double *Q, double *w);

// FP64 path (gemm_f64.hip)
hipError_t gemm1_f64(const Plan &p, int n_fields, const void *rho, int rho_dtype);
hipError_t gemm2_f64(const Plan &p, int n_fields, void *phi, int phi_dtype);
// separable method: the moments (phi transform; theta contraction and
// rotation into Bpart plane 0) and the expansion (rotation and theta
// contraction; phi transform)
hipError_t sep_phi_moments(const Plan &p, int n_fields, const void *rho, int rho_dtype);
hipError_t sep_theta_moments(const Plan &p, int n_fields);
hipError_t sep_theta_expansion(const Plan &p, int n_fields);
hipError_t sep_phi_expansion(const Plan &p, int n_fields, void *phi, int phi_dtype);
// expansion = true: the arguments of GEMM2 (they differ from GEMM1's only
// for the per-patch method, whose GEMM1 sees single-patch fields)
F64Args f64_args(const Plan &p, int n_fields, const void *rho, void *phi, int io_dtype, bool expansion = false);
hipError_t batch_gemm1_f64(const F64Args *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                           int blocks, hipStream_t s);
hipError_t batch_gemm2_f64(const F64Args *args, const BatchItem *items, int n_items, int *head, int io_dtype,
                           int blocks, BatchTrack track, hipStream_t s);

// the choices one field of a plan takes in a batched solve (batch.hip)
struct BatchChoice {
    int splitk, chunks, gemm1_rows, gemm2_rows;
};
BatchChoice batch_choice(const Plan &p);

// radial scans (scan.hip): Bpart -> Bred, M (and the split copies of M)
hipError_t radial_scan(const Plan &p, int n_fields, bool split_out);
ScanArgs scan_args(const Plan &p, int n_fields, bool split_out);
hipError_t batch_scan(const ScanArgs *args, const BatchItem *items, int n_items, int *head, int blocks,
                      hipStream_t s);

// split-BF16 path (gemm_bf16.hip)
hipError_t split_input_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype);
hipError_t gemm1_bf16(const Plan &p, int n_fields, const void *rho, int rho_dtype);
hipError_t gemm2_bf16(const Plan &p, int n_fields, void *phi, int phi_dtype);
// threads of the input split of n_fields fields of a plan
size_t split_input_threads(const Plan &p, int n_fields);
SplitArgs split_args(const Plan &p, int n_fields, const void *rho, void *phi, int io_dtype, bool expansion = false);
// the whole split-form batch in one persistent kernel (items of every stage
// of every field in one queue; see batch_order.h)
hipError_t batch_fused_bf16(const SplitArgs *args, const ScanArgs *sargs, const FusedItem *items, int n_items,
                            FusedCtl ctl, int io_dtype, int blocks, hipStream_t s);

// batched solve (batch.hip)
hipError_t potential_batch(const std::vector<const Plan *> &plans, const void *const *rho, void *const *phi,
                           int dtype, hipStream_t stream);
void forget_plan(const Plan *p);
// per-field completion times (ms from the batch's start) of the last
// batched solve of these plans with this dtype; hipErrorNotFound if none
hipError_t batch_field_times(const std::vector<const Plan *> &plans, int dtype, double *ms);
// K splits used for n_fields fields of a plan (autotuned or heuristic)
int choose_splitk(const Plan &p, int n_fields);

// permuted [rows][np] -> real index [rows][n_lm]
hipError_t unpermute(const Plan &p, int n_fields, const double *src, double *dst);

}  // namespace mpg

// The opaque handle of the C ABI is the plan itself.
struct mpg_plan_s : mpg::Plan {};
