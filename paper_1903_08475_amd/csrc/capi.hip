// C ABI of the library (declared in include/mpg.h): plan creation with
// validation, the solve entry points and error reporting.  Every entry point
// catches its own failures and returns a status; nothing throws across the
// ABI.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "mpg_internal.h"

namespace mpg {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

namespace {

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

// Reports a failed HIP call and clears the thread's last HIP error, which
// would otherwise be returned by later error checks (this library's after
// its launches, or the caller's) although those calls succeeded.
int hip_fail(hipError_t e, const char *where) {
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? MPG_ENOMEM : MPG_EDEVICE;
}

void rot(const double *e, double R[9]) {
    double ca = cos(e[0]), sa = sin(e[0]), cb = cos(e[1]), sb = sin(e[1]), cg = cos(e[2]), sg = sin(e[2]);
    R[0] = ca * cb * cg - sa * sg;  R[1] = sa * cb * cg + ca * sg;  R[2] = -sb * cg;
    R[3] = -ca * cb * sg - sa * cg; R[4] = -sa * cb * sg + ca * cg; R[5] = sb * sg;
    R[6] = ca * sb;                 R[7] = sa * sb;                 R[8] = cb;
}

int roundup(int x, int m) { return (x + m - 1) / m * m; }

// Record an event pair around one stage when timing is on; returns the stop
// event to record after the launch (or nullptr).
hipEvent_t stage_begin(const Plan &p, int stage) {
    if (!p.timing) return nullptr;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return nullptr;
    }
    (void)hipEventRecord(a, p.stream);
    p.events[stage]->push_back(a);
    p.events[stage]->push_back(b);
    return b;
}

void stage_end(const Plan &p, hipEvent_t b) {
    if (b) (void)hipEventRecord(b, p.stream);
}

void clear_events(Plan *p) {
    for (int s = 0; s < 4; ++s)
        if (p->events[s]) {
            for (hipEvent_t e : *p->events[s]) (void)hipEventDestroy(e);
            p->events[s]->clear();
        }
}

void free_plan(mpg_plan_s *p) {
    if (!p) return;
    forget_plan(p);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    void *bufs[] = {p->col_src, p->col_l,  p->Ut,     p->Qt,     p->coef,   p->w,      p->Us,
                    p->Qs,      p->Bpart,  p->Bred,   p->M,      p->Ms,     p->A_split, p->sep_m,
                    p->sep_coff, p->sep_cslot, p->sep_f1, p->sep_t1, p->sep_t2, p->sep_f2, p->sep_F,
                    p->sep_A,   p->sep_kxy, p->sep_xoff, p->sep_perm, p->sep_x1, p->sep_x2,
                    p->sep_f1s, p->sep_f2s};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    clear_events(p);
    for (int s = 0; s < 4; ++s) delete p->events[s];
    delete p;
}

}  // namespace

// K splits of the moment contraction for n_fields fields: the autotuned
// choice if there is one, else enough blocks to cover the chip; never more
// than the plan's work space holds.
// Block shape of a contraction from the timings of its two shapes (t1:
// 128 x 256, t2: 256 x 128) and their block counts b1, b2 (padding
// included), on a chip of `cus` CUs (one block each at a time).  Each
// shape's cost is its chip work: the time of one of its blocks (its time
// over its waves of blocks) times its blocks, over the CUs.  For a solve
// that fills the chip in whole waves that is its time; otherwise it leaves
// out the CUs a partial wave leaves idle, which the other work beside it
// (the fields of a batch) can use.  The cheaper shape is kept when it is
// at least 1% cheaper; else the one with fewer blocks, and the first when
// those are equal too.
static double chip_work(float t, long blocks, int cus) {
    const long waves = (blocks + cus - 1) / cus;
    return waves > 0 ? (double)t * blocks / ((double)waves * cus) : 0.0;
}

static int pick_shape(float t1, float t2, long b1, long b2, int cus) {
    const double c1 = chip_work(t1, b1, cus), c2 = chip_work(t2, b2, cus);
    if (c2 < 0.99 * c1) return 2;
    if (c1 < 0.99 * c2) return 1;
    return b2 < b1 ? 2 : 1;
}

int choose_splitk(const Plan &p, int n_fields) {
    int s;
    if (p.splitk_sel > 0) {
        s = p.splitk_sel;
    } else {
        int col_tiles = p.fold ? (p.ne_p + 63) / 64 + (p.no_p + 63) / 64 : (p.np + 63) / 64;
        int row_tiles = (n_fields * p.n_r + 63) / 64;
        int tiles = col_tiles * row_tiles;
        s = (1024 + tiles - 1) / tiles;
    }
    if (s > p.splitk) s = p.splitk;
    if (s < 1) s = 1;
    return s;
}

}  // namespace mpg

using namespace mpg;

extern "C" {

const char *mpg_last_error(void) { return g_err.c_str(); }

int mpg_plan(const mpg_grid *g, int lmax, int precision, int max_fields, void *stream, mpg_plan_t *out) {
    return mpg_plan_method(g, lmax, precision, max_fields, MPG_METHOD_GLOBAL, stream, out);
}

int mpg_plan_method(const mpg_grid *g, int lmax, int precision, int max_fields, int method, void *stream,
                    mpg_plan_t *out) {
    if (!out) return fail(MPG_EINVAL, "mpg_plan: out is NULL");
    if (method != MPG_METHOD_GLOBAL && method != MPG_METHOD_PER_PATCH && method != MPG_METHOD_SEPARABLE)
        return fail(MPG_EINVAL, "mpg_plan: unknown method");
    *out = nullptr;
    if (!g) return fail(MPG_EINVAL, "mpg_plan: grid is NULL");
    if (g->n_patches < 1 || g->n_patches > MPG_MAX_PATCHES)
        return fail(MPG_EINVAL, "mpg_plan: n_patches outside [1, MPG_MAX_PATCHES]");
    if (g->n_r < 1 || g->n_theta < 1 || g->n_phi < 1) return fail(MPG_EINVAL, "mpg_plan: empty grid");
    if ((long long)g->n_theta * g->n_phi > (1 << 26)) return fail(MPG_EINVAL, "mpg_plan: too many angular cells");
    if (!g->r_edges || !g->euler) return fail(MPG_EINVAL, "mpg_plan: r_edges/euler is NULL");
    if (!(g->r_edges[0] >= 0.0)) return fail(MPG_EINVAL, "mpg_plan: r_edges[0] < 0");
    for (int i = 0; i < g->n_r; ++i)
        if (!(g->r_edges[i + 1] > g->r_edges[i]) || !std::isfinite(g->r_edges[i + 1]))
            return fail(MPG_EINVAL, "mpg_plan: r_edges must increase strictly");
    if (!(g->dtheta > 0.0) || !(g->dphi > 0.0)) return fail(MPG_EINVAL, "mpg_plan: non-positive spacing");
    if (g->theta0 < -1e-12 || g->theta0 + g->n_theta * g->dtheta > M_PI + 1e-12)
        return fail(MPG_EINVAL, "mpg_plan: colatitudes outside [0, pi]");
    if (lmax < 0 || lmax > 64) return fail(MPG_EINVAL, "mpg_plan: lmax outside [0, 64]");
    if (precision != MPG_FP64 && precision != MPG_SPLIT_BF16 && precision != MPG_SPLIT_BF16_TIERED)
        return fail(MPG_EINVAL, "mpg_plan: bad precision");
    if (max_fields < 1 || max_fields > 4096) return fail(MPG_EINVAL, "mpg_plan: max_fields outside [1, 4096]");
    if (g->eval_point != MPG_EVAL_UPPER_VERTEX && g->eval_point != MPG_EVAL_ANGULAR_CENTRE)
        return fail(MPG_EINVAL, "mpg_plan: bad eval_point");
    for (int i = 0; i < 3 * g->n_patches; ++i)
        if (!std::isfinite(g->euler[i])) return fail(MPG_EINVAL, "mpg_plan: non-finite Euler angle");

    mpg_plan_s *p = new (std::nothrow) mpg_plan_s();
    if (!p) return fail(MPG_ENOMEM, "mpg_plan: host allocation");
    p->n_patches = g->n_patches;
    p->n_r = g->n_r;
    p->n_theta = g->n_theta;
    p->n_phi = g->n_phi;
    p->n_ang = g->n_theta * g->n_phi;
    p->theta0 = g->theta0;
    p->phi0 = g->phi0;
    p->dtheta = g->dtheta;
    p->dphi = g->dphi;
    p->lmax = lmax;
    p->n_lm = (lmax + 1) * (lmax + 1);
    p->precision = precision;
    p->max_fields = max_fields;
    p->G = g->G;
    p->eval_centre = g->eval_point == MPG_EVAL_ANGULAR_CENTRE;
    p->stream = (hipStream_t)stream;
    p->per_patch = method == MPG_METHOD_PER_PATCH;
    (void)hipGetDevice(&p->device);

    if (g->n_patches == 2) {
        // fold: patch 1 is patch 0 turned by pi about the common z axis
        double R0[9], R1[9];
        rot(g->euler, R0);
        rot(g->euler + 3, R1);
        const double D[3] = {-1.0, -1.0, 1.0};
        double dev = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) dev = fmax(dev, fabs(R1[3 * i + j] - D[i] * R0[3 * i + j]));
        p->fold = dev <= 1e-12 && !p->per_patch;
        // per-patch weights can only be folded when both patches carry the same
        if (p->fold && g->overlap_w && g->w_per_patch) {
            const size_t n = (size_t)g->n_theta * g->n_phi;
            for (size_t c = 0; c < n && p->fold; ++c) p->fold = g->overlap_w[c] == g->overlap_w[n + c];
        }
        if (!g->overlap_w) {
            // overlap weights need the Yin<->Yang relation R0^T R1 = P and
            // extents symmetric about the patch centre
            const double P[9] = {-1, 0, 0, 0, 0, 1, 0, 1, 0};
            double d2 = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k) s += R0[3 * k + i] * R1[3 * k + j];
                    d2 = fmax(d2, fabs(s - P[3 * i + j]));
                }
            double th_hi = g->theta0 + g->n_theta * g->dtheta, ph_hi = g->phi0 + g->n_phi * g->dphi;
            bool sym = fabs(g->theta0 + th_hi - M_PI) < 1e-12 && fabs(g->phi0 + ph_hi) < 1e-12 &&
                       g->theta0 >= 0.0 && g->theta0 < 0.5 * M_PI && ph_hi >= 0.5 * M_PI - 1e-15 &&
                       ph_hi <= M_PI + 1e-12;
            if (d2 > 1e-12 || !sym) {
                free_plan(p);
                return fail(MPG_EUNSUPPORTED,
                            "mpg_plan: overlap weights are computed only for the Yin<->Yang relation with symmetric "
                            "extents; pass overlap_w");
            }
            p->ovl_sc = cos(g->theta0);
            p->ovl_kap_inf = ph_hi >= M_PI - 1e-15;
            p->ovl_kap = p->ovl_kap_inf ? 0.0 : 1.0 / tan(M_PI - ph_hi);
        }
    }

    if (g->n_patches > 2 && !g->overlap_w) {
        free_plan(p);
        return fail(MPG_EUNSUPPORTED, "mpg_plan: more than two patches need overlap_w");
    }
    if (p->per_patch && g->overlap_w && g->w_per_patch) {
        // one local table U serves every patch: the weights must agree
        const size_t n = (size_t)g->n_theta * g->n_phi;
        for (size_t c = 0; c < n * g->n_patches; ++c)
            if (g->overlap_w[c] != g->overlap_w[c % n]) {
                free_plan(p);
                return fail(MPG_EUNSUPPORTED, "mpg_plan: the per-patch method needs one weight set for all patches");
            }
    }
    p->npat = (p->fold || p->per_patch) ? 1 : g->n_patches;
    if (method == MPG_METHOD_SEPARABLE) {
        // grid limits of its launches: theta rows and 128-row blocks of
        // (field, patch, shell) rows on a grid axis, a weight row in LDS
        const long long vblocks = ((long long)max_fields * g->n_patches * g->n_r + 127) / 128;
        const char *why = precision == MPG_SPLIT_BF16_TIERED ? "the separable method takes MPG_FP64 or MPG_SPLIT_BF16"
                          : (g->n_theta > 65535 || vblocks > 65535 || g->n_phi > 8192)
                              ? "the separable method takes at most 65535 theta rows, 8192 phi cells and 65535 "
                                "blocks of 128 (field, patch, shell) rows"
                              : nullptr;
        if (why) {
            free_plan(p);
            return fail(MPG_EUNSUPPORTED, std::string("mpg_plan: ") + why);
        }
        p->sep = true;
    }

    // column layout
    if (p->fold) {
        int ne = 0;
        for (int l = 0; l <= lmax; ++l)
            for (int m = 0; m <= l; m += 2) ne += (m == 0 ? 1 : 2);
        p->n_e = ne;
        p->n_o = p->n_lm - ne;
        p->ne_p = roundup(p->n_e, kColPad);
        p->no_p = roundup(p->n_o, kColPad);
    } else {
        p->n_e = p->n_lm;
        p->n_o = 0;
        p->ne_p = roundup(p->n_lm, kColPad);
        p->no_p = 0;
    }
    p->np = p->ne_p + p->no_p;
    p->np_alloc = p->np + kColSlack;
    p->n_angp = roundup(p->n_ang, kAngPad);
    if (p->sep) {
        // phi columns: the order-0 column, then C and S of the orders 1..lmax
        // in tiles of 16 (at least one each); the mirror fold on a phi grid
        // symmetric about 0 with an even cell count
        const int n = p->n_phi;
        p->sep_ce = std::max(16, roundup(lmax, 16));
        p->sep_co = p->sep_ce;
        p->sep_lp = roundup(lmax + 1, 16);
        p->sep_mir = n % 2 == 0 && fabs(p->phi0 + 0.5 * n * p->dphi) <= 1e-12;
        p->sep_kh = p->sep_mir ? n / 2 : n;
        p->sep_khp = roundup(p->sep_kh, 16);
        p->sep_kx = !p->sep_mir ? n : p->eval_centre ? n / 2 : n / 2 + 1;
        p->sep_nt2 = std::max(1, (lmax + 31) / 32);
        p->sep_kxp = roundup(p->sep_kx, 64);
    }

    // work space
    {
        int col_tiles = p->fold ? (p->ne_p + 63) / 64 + (p->no_p + 63) / 64 : (p->np + 63) / 64;
        int tiles = col_tiles * ((p->n_r + 63) / 64);
        int s = (1024 + tiles - 1) / tiles;
        int kmax = p->kang() / 64;
        // room for at least four splits for the autotuner to try, while the
        // partial sums stay within 2 GiB, and up to 32 (small grids, whose
        // moment contraction fills the chip only when split finely) while
        // they stay within 512 MiB
        const double plane = 8.0 * p->np * (double)p->vfields(max_fields) * p->n_r;
        while (s < 4 && (s + 1) * plane <= 2147483648.0) ++s;
        while (s < 32 && (s + 1) * plane <= 536870912.0) ++s;
        p->splitk = s < 1 ? 1 : (s > kmax ? kmax : s);
        if (p->splitk < 1) p->splitk = 1;
    }
    size_t rows = (size_t)p->rows_alloc();
    hipError_t e;
    if ((e = hipMalloc(&p->Bpart, sizeof(double) * p->splitk * rows * p->np)) != hipSuccess ||
        (e = hipMalloc(&p->Bred, sizeof(double) * rows * p->np)) != hipSuccess ||
        (e = hipMalloc(&p->M, sizeof(double) * rows * p->np)) != hipSuccess) {
        int rc = hip_fail(e, "mpg_plan: work space");
        free_plan(p);
        return rc;
    }
    if (precision == MPG_SPLIT_BF16_TIERED) {
        // leading columns of each block up to degree MPG_TIER_LMAX (columns
        // keep the order of the real index inside a block), rounded up to K slabs
        int ce = 0, co = 0;
        for (int l = 0; l <= lmax && l <= MPG_TIER_LMAX; ++l)
            for (int m = 0; m <= l; ++m) {
                const int c = m == 0 ? 1 : 2;
                if (!p->fold || m % 2 == 0) ce += c;
                else co += c;
            }
        p->six_e = std::min(roundup(ce, kSlabK), p->ne_p);
        p->six_o = std::min(roundup(co, kSlabK), p->no_p);
    } else {
        p->six_e = p->ne_p;
        p->six_o = p->no_p;
    }
    if (p->split()) {
        // tile-slab blocks; rows past the last field stay zero (finite)
        const size_t nM = (size_t)p->out_row_tiles() * (p->kq() / kSlabK) * 3 * kBlk;
        const size_t nA = (size_t)(p->fold ? 2 : 1) * p->row_tiles() * (p->kang() / kSlabK) * 3 * kBlk;
        if ((e = hipMalloc(&p->Ms, sizeof(bf16) * nM)) != hipSuccess ||
            (e = hipMalloc(&p->A_split, sizeof(bf16) * nA)) != hipSuccess ||
            (e = hipMemset(p->Ms, 0, sizeof(bf16) * nM)) != hipSuccess ||
            (e = hipMemset(p->A_split, 0, sizeof(bf16) * nA)) != hipSuccess) {
            int rc = hip_fail(e, "mpg_plan: split work space");
            free_plan(p);
            return rc;
        }
    }
    if (p->sep) {
        // zeroed once so that no padding row ever holds a non-finite value
        const size_t n = (size_t)p->sep_nc() * p->n_theta * p->sep_ldv(), na = (size_t)p->n_lm * p->sep_ldv();
        if ((e = hipMalloc(&p->sep_F, sizeof(double) * n)) != hipSuccess ||
            (e = hipMemset(p->sep_F, 0, sizeof(double) * n)) != hipSuccess ||
            (e = hipMalloc(&p->sep_A, sizeof(double) * na)) != hipSuccess ||
            (e = hipMemset(p->sep_A, 0, sizeof(double) * na)) != hipSuccess) {
            int rc = hip_fail(e, "mpg_plan: separable work space");
            free_plan(p);
            return rc;
        }
    }
    if ((e = build_tables(*p, g->euler, g->r_edges, g->overlap_w, g->w_per_patch)) != hipSuccess) {
        int rc = hip_fail(e, "mpg_plan: table build");
        free_plan(p);
        return rc;
    }
    *out = p;
    return MPG_OK;
}

static int check_call(mpg_plan_t p, int n_fields, const void *rho, int dt, const char *who) {
    if (!p) return fail(MPG_EINVAL, std::string(who) + ": plan is NULL");
    if (n_fields < 1 || n_fields > p->max_fields)
        return fail(MPG_EINVAL, std::string(who) + ": n_fields outside [1, max_fields]");
    if (!rho) return fail(MPG_EINVAL, std::string(who) + ": rho is NULL");
    if (dt != MPG_F64 && dt != MPG_F32) return fail(MPG_EINVAL, std::string(who) + ": bad dtype");
    return MPG_OK;
}

// GEMM1 and the scans of n_fields fields (for the per-patch method:
// n_patches single-patch fields per field, each patch in its own frame).
// all_six: the split forms take six products on every moment column (the
// moments a caller reads back meet the six-product error bound in either
// split form; the tiered form's three-product columns only feed the
// expansion).
static int run_moments(const Plan *p, int n_fields_in, const void *rho, int rho_dtype, bool split_out,
                       bool all_six = false) {
    hipError_t e;
    const int n_fields = p->vfields(n_fields_in);
    int sk = p->sep ? 1 : choose_splitk(*p, n_fields);
    Plan q = *p;
    q.splitk = sk;
    if (all_six) {
        q.six_e = q.ne_p;
        q.six_o = q.no_p;
    }
    hipEvent_t ev;
    if (p->sep) {
        // phi transform; theta contraction and rotation (into partial plane 0); radial scans
        ev = stage_begin(q, 0);
        e = sep_phi_moments(q, n_fields, rho, rho_dtype);
        stage_end(q, ev);
        if (e != hipSuccess) return hip_fail(e, "phi transform");
        ev = stage_begin(q, 1);
        e = sep_theta_moments(q, n_fields);
        stage_end(q, ev);
        if (e != hipSuccess) return hip_fail(e, "theta contraction and rotation");
        ev = stage_begin(q, 2);
        e = radial_scan(q, n_fields, false);
        stage_end(q, ev);
        if (e != hipSuccess) return hip_fail(e, "radial scan");
        return MPG_OK;
    }
    if (p->split()) {
        ev = stage_begin(q, 0);
        e = split_input_bf16(q, n_fields, rho, rho_dtype);
        stage_end(q, ev);
        if (e != hipSuccess) return hip_fail(e, "input split");
    }
    ev = stage_begin(q, 1);
    if (p->split())
        e = gemm1_bf16(q, n_fields, rho, rho_dtype);
    else
        e = gemm1_f64(q, n_fields, rho, rho_dtype);
    stage_end(q, ev);
    if (e != hipSuccess) return hip_fail(e, "moment contraction");
    ev = stage_begin(q, 2);
    e = radial_scan(q, n_fields, split_out);
    stage_end(q, ev);
    if (e != hipSuccess) return hip_fail(e, "radial scan");
    return MPG_OK;
}

int mpg_moments(mpg_plan_t p, int n_fields, const void *rho, int rho_dtype, double *B, double *M) {
    int rc = check_call(p, n_fields, rho, rho_dtype, "mpg_moments");
    if (rc) return rc;
    if ((rc = run_moments(p, n_fields, rho, rho_dtype, false, true))) return rc;
    hipError_t e;
    const int vf = p->vfields(n_fields);
    if (B && (e = unpermute(*p, vf, p->Bred, B)) != hipSuccess) return hip_fail(e, "mpg_moments: B");
    if (M && (e = unpermute(*p, vf, p->M, M)) != hipSuccess) return hip_fail(e, "mpg_moments: M");
    return MPG_OK;
}

static int solve(const Plan *p, int n_fields, const void *rho, int rho_dtype, void *phi, int phi_dtype) {
    int rc;
    bool split = p->split();
    if ((rc = run_moments(p, n_fields, rho, rho_dtype, split))) return rc;
    hipEvent_t ev;
    hipError_t e;
    if (p->sep) {
        // rotation and theta contraction (timed with the moments' ones), phi transform
        ev = stage_begin(*p, 1);
        e = sep_theta_expansion(*p, n_fields);
        stage_end(*p, ev);
        if (e != hipSuccess) return hip_fail(e, "expansion");
        ev = stage_begin(*p, 3);
        e = sep_phi_expansion(*p, n_fields, phi, phi_dtype);
    } else {
        ev = stage_begin(*p, 3);
        e = split ? gemm2_bf16(*p, n_fields, phi, phi_dtype) : gemm2_f64(*p, n_fields, phi, phi_dtype);
    }
    stage_end(*p, ev);
    if (e != hipSuccess) return hip_fail(e, "expansion");
    return MPG_OK;
}

int mpg_potential(mpg_plan_t p, int n_fields, const void *rho, int rho_dtype, void *phi, int phi_dtype) {
    int rc = check_call(p, n_fields, rho, rho_dtype, "mpg_potential");
    if (rc) return rc;
    if (!phi) return fail(MPG_EINVAL, "mpg_potential: phi is NULL");
    if (phi_dtype != MPG_F64 && phi_dtype != MPG_F32) return fail(MPG_EINVAL, "mpg_potential: bad phi dtype");
    return solve(p, n_fields, rho, rho_dtype, phi, phi_dtype);
}

// ---- the solve without allocation (mpg_potential_static) -----------------
//
// Work space of mpg_potential_static: one file-scope device array per GPU
// the library runs on, held until the process ends.  In host code its name
// is a stand-in, not a device address: the address is taken per device
// with hipGetSymbolAddress (with that device current) on the first call on
// the device, and only that address is handed to kernels.
}  // extern "C"

namespace mpg {
namespace {

constexpr size_t kStaticBytes = size_t(MPG_STATIC_WORKSPACE_MB) << 20;
__device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's scratch array (taken once per device)
hipError_t scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets of the work arrays of one call (q sized for this call's
// fields: q.max_fields = n_fields) with `splitk` K splits: Bpart, Bred, M,
// and for the split forms Ms and A_split; returns the total.
size_t static_layout(const Plan &q, int splitk, size_t off[5]) {
    const size_t rows = (size_t)q.rows_alloc(), np = (size_t)q.np;
    size_t o = 0;
    off[0] = o;
    o += align256(sizeof(double) * splitk * rows * np);
    off[1] = o;
    o += align256(sizeof(double) * rows * np);
    off[2] = o;
    o += align256(sizeof(double) * rows * np);
    off[3] = off[4] = o;
    if (q.split()) {
        o += align256(sizeof(bf16) * (size_t)q.out_row_tiles() * (q.kq() / kSlabK) * 3 * kBlk);
        off[4] = o;
        o += align256(sizeof(bf16) * (size_t)(q.fold ? 2 : 1) * q.row_tiles() * (q.kang() / kSlabK) * 3 * kBlk);
    }
    return o;
}

}  // namespace
}  // namespace mpg

extern "C" {

int mpg_potential_static(mpg_plan_t p, int n_fields, const void *rho, int rho_dtype, void *phi, int phi_dtype) {
    int rc = check_call(p, n_fields, rho, rho_dtype, "mpg_potential_static");
    if (rc) return rc;
    if (p->sep) return fail(MPG_EUNSUPPORTED, "mpg_potential_static: separable-method plans need their work array");
    if (!phi) return fail(MPG_EINVAL, "mpg_potential_static: phi is NULL");
    if (phi_dtype != MPG_F64 && phi_dtype != MPG_F32)
        return fail(MPG_EINVAL, "mpg_potential_static: bad phi dtype");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "mpg_potential_static");
    if (dev != p->device) return fail(MPG_EINVAL, "mpg_potential_static: the plan's device must be current");
    if (dev < 0 || dev >= kMaxDevices) return fail(MPG_EUNSUPPORTED, "mpg_potential_static: device index too large");
    // this call's arrays, with the plan's K split choice reduced until they fit
    Plan q = *p;
    q.max_fields = n_fields;
    q.timing = false;  // stage events would be created (allocated) per call
    int sk = choose_splitk(q, q.vfields(n_fields));
    size_t off[5];
    while (sk > 1 && static_layout(q, sk, off) > kStaticBytes) --sk;
    const size_t need = static_layout(q, sk, off);
    if (need > kStaticBytes)
        return fail(MPG_EINVAL, "mpg_potential_static: the call needs " + std::to_string(need >> 20) +
                                    " MiB of work space, more than the " +
                                    std::to_string(MPG_STATIC_WORKSPACE_MB) + " MiB static work space");
    void *base = nullptr;
    if ((e = scratch_address(dev, &base)) != hipSuccess) return hip_fail(e, "mpg_potential_static: work space");
    unsigned char *b = (unsigned char *)base;
    q.splitk = sk;
    q.splitk_sel = sk;
    q.Bpart = (double *)(b + off[0]);
    q.Bred = (double *)(b + off[1]);
    q.M = (double *)(b + off[2]);
    q.Ms = q.split() ? (bf16 *)(b + off[3]) : nullptr;
    q.A_split = q.split() ? (bf16 *)(b + off[4]) : nullptr;
    return solve(&q, n_fields, rho, rho_dtype, phi, phi_dtype);
}

int mpg_potential_batch(int n, const mpg_plan_t *plans, const void *const *rho, void *const *phi, int dtype) {
    if (n < 1 || !plans || !rho || !phi) return fail(MPG_EINVAL, "mpg_potential_batch: bad arguments");
    if (dtype != MPG_F64 && dtype != MPG_F32) return fail(MPG_EINVAL, "mpg_potential_batch: bad dtype");
    std::vector<const Plan *> ps(n);
    for (int f = 0; f < n; ++f) {
        if (!plans[f]) return fail(MPG_EINVAL, "mpg_potential_batch: NULL plan");
        if (!rho[f] || !phi[f]) return fail(MPG_EINVAL, "mpg_potential_batch: NULL field");
        if (plans[f]->precision != plans[0]->precision)
            return fail(MPG_EINVAL, "mpg_potential_batch: plans differ in precision");
        if (plans[f]->per_patch)
            return fail(MPG_EUNSUPPORTED, "mpg_potential_batch: per-patch-method plans are solved one by one");
        if (plans[f]->sep)
            return fail(MPG_EUNSUPPORTED, "mpg_potential_batch: separable-method plans are solved one by one");
        for (int g = 0; g < f; ++g)
            if (plans[g] == plans[f])
                return fail(MPG_EINVAL, "mpg_potential_batch: a plan appears twice (they own their work space)");
        ps[f] = plans[f];
    }
    hipError_t e = potential_batch(ps, rho, phi, dtype, plans[0]->stream);
    if (e != hipSuccess) return hip_fail(e, "mpg_potential_batch");
    return MPG_OK;
}

int mpg_batch_field_times(int n, const mpg_plan_t *plans, int dtype, double *ms) {
    if (n < 1 || !plans || !ms) return fail(MPG_EINVAL, "mpg_batch_field_times: bad arguments");
    std::vector<const Plan *> ps(n);
    for (int f = 0; f < n; ++f) {
        if (!plans[f]) return fail(MPG_EINVAL, "mpg_batch_field_times: NULL plan");
        ps[f] = plans[f];
    }
    hipError_t e = batch_field_times(ps, dtype, ms);
    if (e == hipErrorNotFound) return fail(MPG_EINVAL, "mpg_batch_field_times: no batched solve of these plans");
    if (e == hipErrorLaunchTimeOut)
        return fail(MPG_EDEVICE, "mpg_batch_field_times: a stage wait of the last batched solve gave up; its "
                                 "results are incomplete");
    if (e != hipSuccess) return hip_fail(e, "mpg_batch_field_times");
    return MPG_OK;
}

int mpg_batch_choices(int n, const mpg_plan_t *plans, int dtype, int *splitk, int *chunks, int *gemm1_rows,
                      int *gemm2_rows) {
    if (n < 1 || !plans) return fail(MPG_EINVAL, "mpg_batch_choices: bad arguments");
    if (dtype != MPG_F64 && dtype != MPG_F32) return fail(MPG_EINVAL, "mpg_batch_choices: bad dtype");
    for (int f = 0; f < n; ++f) {
        if (!plans[f]) return fail(MPG_EINVAL, "mpg_batch_choices: NULL plan");
        BatchChoice c = batch_choice(*plans[f]);
        if (splitk) splitk[f] = c.splitk;
        if (chunks) chunks[f] = c.chunks;
        if (gemm1_rows) gemm1_rows[f] = c.gemm1_rows;
        if (gemm2_rows) gemm2_rows[f] = c.gemm2_rows;
    }
    return MPG_OK;
}

int mpg_autotune(mpg_plan_t p, int n_fields_in, const void *rho, int rho_dtype, int *splitk, int *chunks,
                 int *gemm1_rows, int *gemm2_rows) {
    int rc = check_call(p, n_fields_in, rho, rho_dtype, "mpg_autotune");
    if (rc) return rc;
    if (p->sep) return fail(MPG_EUNSUPPORTED, "mpg_autotune: the separable method has no choices to tune");
    const int n_fields = p->vfields(n_fields_in);
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "mpg_autotune");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "mpg_autotune");
    }
    const bool split = p->split();
    // Every timing takes kRounds rounds, each launching every candidate once
    // (round 0 is a warm-up), and keeps each candidate's fastest: clock
    // changes during the tuning then weigh on all candidates alike.
    constexpr int kRounds = 4;
    auto time_once = [&](const Plan &q, int what, void *phi, float *ms) -> hipError_t {
        hipError_t err;
        if ((err = hipEventRecord(a, q.stream)) != hipSuccess) return err;
        if (what == 0) err = split ? gemm1_bf16(q, n_fields, rho, rho_dtype) : gemm1_f64(q, n_fields, rho, rho_dtype);
        else if (what == 1) err = radial_scan(q, n_fields, split);
        else err = gemm2_bf16(q, n_fields_in, phi, rho_dtype);
        if (err != hipSuccess) return err;
        if ((err = hipEventRecord(b, q.stream)) != hipSuccess) return err;
        if ((err = hipEventSynchronize(b)) != hipSuccess) return err;
        return hipEventElapsedTime(ms, a, b);
    };
    // index of the fastest candidate: the first, unless another is at least
    // 1% faster than the best so far
    auto keep_within_1pct = [](const std::vector<float> &t) {
        size_t k = 0;
        for (size_t i = 1; i < t.size(); ++i)
            if (t[i] < 0.99f * t[k]) k = i;
        return k;
    };
    if (split && (e = split_input_bf16(*p, n_fields, rho, rho_dtype)) != hipSuccess) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return hip_fail(e, "mpg_autotune");
    }
    // Moment contraction: every (block shape, K split) pair, timed as the
    // contraction plus the scan that reduces its partial sums.  Shapes:
    // split forms 128 x 256 (1, the default) or 256 x 128 (2); FP64 tiles
    // of 128 x 128 (1) or 64 x 64 (2).  K splits: the heuristic choice,
    // then 1, 2, 3, 4 and powers of two up to the work space.
    std::vector<int> cands;
    Plan unset = *p;  // the heuristic choice (the plan keeps its choices until the tuning succeeds)
    unset.splitk_sel = 0;
    const int heur = choose_splitk(unset, n_fields);
    cands.push_back(heur);
    for (int s = 1; s <= p->splitk; s = s < 4 ? s + 1 : 2 * s)  // 1, 2, 3, 4, 8, 16, ...
        if (s != heur) cands.push_back(s);
    size_t one = 0;  // index of K split 1
    while (cands[one] != 1) ++one;
    std::vector<float> tk[3], tg1[3];  // [shape][split]: contraction + scan; contraction alone
    for (int r = 1; r <= 2; ++r) {
        tk[r].assign(cands.size(), 1e30f);
        tg1[r].assign(cands.size(), 1e30f);
    }
    for (int round = 0; round < kRounds && e == hipSuccess; ++round)
        for (int r = 1; r <= 2 && e == hipSuccess; ++r)
            for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
                Plan q = *p;
                q.splitk = cands[i];
                q.gemm1_rows = r;
                float t1 = 0.0f, t2 = 0.0f;
                if ((e = time_once(q, 0, nullptr, &t1)) == hipSuccess &&
                    (e = time_once(q, 1, nullptr, &t2)) == hipSuccess && round > 0) {
                    tk[r][i] = std::min(tk[r][i], t1 + t2);
                    tg1[r][i] = std::min(tg1[r][i], t1);
                }
            }
    // per shape its K split (the heuristic unless another is 1% faster);
    // single solves take the default shape unless the other is 1% faster
    const size_t k1 = keep_within_1pct(tk[1]), k2 = keep_within_1pct(tk[2]);
    const int best_g1 = tk[2][k2] < 0.99f * tk[1][k1] ? 2 : 1;
    const int best_s = cands[best_g1 == 2 ? k2 : k1];
    // rows of the contractions (GEMM1's per-patch rows included)
    const int rt1 = (n_fields * p->n_r + kSplitTile - 1) / kSplitTile;
    const int rt2 = (n_fields_in * p->n_r + kSplitTile - 1) / kSplitTile;
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (cus < 1) cus = 1;
    // batched solves: the shape with less chip work without a K split (a
    // batch splits K its own way, and other fields fill the chip)
    int batch_g1 = best_g1;
    if (e == hipSuccess) {
        long b1, b2;
        if (split) {
            const int ct_e = p->tiles_e(), ct_o = p->tiles_o();
            b1 = (long)((ct_e + 1) / 2 + (ct_o + 1) / 2) * rt1;
            b2 = (long)(ct_e + ct_o) * ((rt1 + 1) / 2);
        } else {
            auto tiles = [&](int t) {
                const int ct = p->fold ? (p->ne_p + t - 1) / t + (p->no_p + t - 1) / t : (p->np + t - 1) / t;
                return (long)ct * ((n_fields * p->n_r + t - 1) / t);
            };
            b1 = tiles(kF64Tile1);
            b2 = tiles(64);
        }
        batch_g1 = pick_shape(tg1[1][one], tg1[2][one], b1, b2, cus);
    }
    int best_c = p->scan_chunks;
    if (e == hipSuccess) {
        // scan schedule: shell chunks per column, on the partial sums of the
        // chosen K split (the scan leaves them in place)
        Plan q = *p;
        q.splitk = best_s;
        q.gemm1_rows = best_g1;
        float t0 = 0.0f;
        e = time_once(q, 0, nullptr, &t0);
        std::vector<int> chs;
        for (int ch : {4, 8, 12, 16})
            if (ch <= p->n_r || ch == 4) chs.push_back(ch);
        std::vector<float> tc(chs.size(), 1e30f);
        for (int round = 0; round < kRounds && e == hipSuccess; ++round)
            for (size_t i = 0; i < chs.size() && e == hipSuccess; ++i) {
                q.scan_chunks = chs[i];
                float t = 0.0f;
                if ((e = time_once(q, 1, nullptr, &t)) == hipSuccess && round > 0) tc[i] = std::min(tc[i], t);
            }
        if (e == hipSuccess) {
            size_t k = 0;
            for (size_t i = 1; i < tc.size(); ++i)
                if (tc[i] < tc[k]) k = i;
            best_c = chs[k];
        }
    }
    int best_r = p->gemm2_rows;
    if (e == hipSuccess && split) {
        // block shape of the expansion, timed on the moments of this input
        // (GEMM1 and the scan with the choices above write M's split copy);
        // Phi goes to a temporary buffer of one call's size (if that cannot
        // be allocated, the shape stays as it is)
        const size_t cells = (size_t)n_fields_in * p->n_patches * p->n_r * p->n_ang;
        void *phi = nullptr;
        if (hipMalloc(&phi, cells * (rho_dtype == MPG_F64 ? sizeof(double) : sizeof(float))) != hipSuccess) {
            (void)hipGetLastError();
            phi = nullptr;
        }
        if (phi) {
            Plan q = *p;
            q.splitk = best_s;
            q.scan_chunks = best_c;
            q.gemm1_rows = best_g1;
            e = gemm1_bf16(q, n_fields, rho, rho_dtype);
            if (e == hipSuccess) e = radial_scan(q, n_fields, true);
            float tr[3] = {0.0f, 1e30f, 1e30f};
            for (int round = 0; round < kRounds && e == hipSuccess; ++round)
                for (int r = 1; r <= 2 && e == hipSuccess; ++r) {
                    q.gemm2_rows = r;
                    float t = 0.0f;
                    if ((e = time_once(q, 2, phi, &t)) == hipSuccess && round > 0) tr[r] = std::min(tr[r], t);
                }
            if (e == hipSuccess) {
                const int at = p->n2() / kSplitTile;
                best_r = pick_shape(tr[1], tr[2], (long)rt2 * ((at + 1) / 2), (long)((rt2 + 1) / 2) * at, cus);
            }
            hipError_t es = hipStreamSynchronize(p->stream);
            hipError_t ef = hipFree(phi);
            if (e == hipSuccess) e = es != hipSuccess ? es : ef;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "mpg_autotune");
    p->splitk_sel = best_s;
    p->scan_chunks = best_c;
    p->gemm1_rows = best_g1;
    p->gemm1_rows_batch = batch_g1;
    p->gemm2_rows = best_r;
    ++p->tune_epoch;
    if (splitk) *splitk = best_s;
    if (chunks) *chunks = best_c;
    if (gemm1_rows) *gemm1_rows = best_g1;
    if (gemm2_rows) *gemm2_rows = split ? best_r : 1;
    return MPG_OK;
}

int mpg_tables(mpg_plan_t p, double *U, double *Q, double *w) {
    if (!p) return fail(MPG_EINVAL, "mpg_tables: plan is NULL");
    hipError_t e = export_tables(*p, U, Q, w);
    if (e != hipSuccess) return hip_fail(e, "mpg_tables");
    return MPG_OK;
}

int mpg_set_tuning(mpg_plan_t p, int splitk, int chunks, int gemm1_rows, int gemm2_rows) {
    if (!p) return fail(MPG_EINVAL, "mpg_set_tuning: plan is NULL");
    if (p->sep) return fail(MPG_EUNSUPPORTED, "mpg_set_tuning: the separable method has no choices to tune");
    if (splitk > p->splitk) return fail(MPG_EINVAL, "mpg_set_tuning: K split exceeds the plan's work space");
    if (chunks > 16) return fail(MPG_EINVAL, "mpg_set_tuning: more than 16 shell chunks");
    if (gemm1_rows > 2) return fail(MPG_EINVAL, "mpg_set_tuning: gemm1_rows must be 1 or 2");
    if (gemm2_rows > 2) return fail(MPG_EINVAL, "mpg_set_tuning: gemm2_rows must be 1 or 2");
    if (splitk > 0) p->splitk_sel = splitk;
    if (chunks > 0) p->scan_chunks = chunks;
    if (gemm1_rows > 0) p->gemm1_rows = p->gemm1_rows_batch = gemm1_rows;
    if (gemm2_rows > 0) p->gemm2_rows = gemm2_rows;
    ++p->tune_epoch;
    return MPG_OK;
}

int mpg_plan_info(mpg_plan_t p, int *n_lm, long long *field_elems) {
    if (!p) return fail(MPG_EINVAL, "mpg_plan_info: plan is NULL");
    if (n_lm) *n_lm = p->n_lm;
    if (field_elems) *field_elems = (long long)p->n_patches * p->n_r * p->n_ang;
    return MPG_OK;
}

int mpg_timing(mpg_plan_t p, int enable) {
    if (!p) return fail(MPG_EINVAL, "mpg_timing: plan is NULL");
    for (int s = 0; s < 4; ++s)
        if (!p->events[s]) {
            p->events[s] = new (std::nothrow) std::vector<hipEvent_t>();
            if (!p->events[s]) return fail(MPG_ENOMEM, "mpg_timing: host allocation");
        }
    p->timing = enable != 0;
    return MPG_OK;
}

int mpg_stage_times(mpg_plan_t p, double ms[4], long long launches[4], int reset) {
    if (!p) return fail(MPG_EINVAL, "mpg_stage_times: plan is NULL");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "mpg_stage_times");
    for (int s = 0; s < 4; ++s) {
        double tot = 0.0;
        long long n = 0;
        if (p->events[s])
            for (size_t k = 0; k + 1 < p->events[s]->size(); k += 2) {
                float t = 0.0f;
                if ((e = hipEventElapsedTime(&t, (*p->events[s])[k], (*p->events[s])[k + 1])) != hipSuccess)
                    return hip_fail(e, "mpg_stage_times");
                tot += t;
                ++n;
            }
        if (ms) ms[s] = tot;
        if (launches) launches[s] = n;
    }
    if (reset) clear_events(p);
    return MPG_OK;
}

int mpg_sync(mpg_plan_t p) {
    if (!p) return fail(MPG_EINVAL, "mpg_sync: plan is NULL");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "mpg_sync");
    return MPG_OK;
}

void mpg_destroy(mpg_plan_t p) { free_plan(p); }

}  // extern "C"
