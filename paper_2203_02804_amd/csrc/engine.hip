// Host side of the pricer: the C ABI, device workspace, and the sweep driver that launches
// the TT-cross kernels for a batch of (option, term) work items.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"
#include "plan.hpp"
#include "ttfp.h"

namespace ttfp {
__global__ void k_init(Item *items, int n_items);
__global__ void k_fiber(Item *items, ItemList work, int t, int dir, int mode);
__global__ void k_eval_points(const Item *items, long long npts, const int *idx, cplx *out);
__global__ void k_tsqr(Item *items, ItemList work, int t, int dir, int level, int BR, int G);
__global__ void k_qrcp(Item *items, ItemList work, int t, int dir, int BR, int G);
template <int W> __global__ void k_gram(Item *items, ItemList work, int t, int dir, int pass);
__global__ void k_chol(Item *items, ItemList work, int t, int dir, int pass, int last);
__global__ void k_xform(Item *items, ItemList work, int t, int dir, int pass);
template <int W, int P> __global__ void k_basis(Item *items, ItemList work, int t, int dir);
__global__ void k_maxvol(Item *items, ItemList work, int t, int dir, int rmax, int warm);
__global__ void k_maxvol_refine(Item *items, ItemList work, int t, int dir, int rmax, int *moved);
__global__ void k_clear_moved(int *moved);
template <int W, int P> __global__ void k_interp(Item *items, ItemList work, int t, int dir, int mode, int bound);
__global__ void k_finish(Item *items, ItemList work, int t, int dir);
__global__ void k_core_sum(Item *items, ItemList work, int t, int dir, int mode);
__global__ void k_contract(Item *items, ItemList work);
__global__ void k_core_moments(Item *items, const int *active);
__global__ void k_moments(Item *items, const int *active, cplx *out, int stride);
__global__ void k_tt_values(const Item *items, int item, long long npts, const int *idx, cplx *out);
__global__ void k_err_est(Item *items, const int *active);
__global__ void k_ladder_weights(const Item *items, int item, int k, int S, const double *dm, cplx *W);
__global__ void k_inner_x(const Item *items, int ia, int ib, int k, const cplx *E, cplx *X);
__global__ void k_inner_e(const Item *items, int ia, int ib, int k, const cplx *X, cplx *E);
__global__ void k_ladder_core(const Item *items, int item, int k, int S, const cplx *W, cplx *T);
__global__ void k_ladder_chain(const Item *items, int item, int k, int S, const cplx *T, cplx *V);
__global__ void k_converge(const Item *items, int *active, OptState *os, int n_opts, const double *item_scale, int *flags);
}  // namespace ttfp

using namespace ttfp;

struct ttfp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    // grow-only device arena for item buffers
    char *arena = nullptr;
    size_t arena_bytes = 0;
    Item *d_items = nullptr;
    size_t items_cap = 0;
    int *d_active = nullptr;
    cplx *d_moments = nullptr;
    size_t moments_cap = 0;
    // last single-option call (for ttfp_tt_values)
    std::vector<Item> last_items;
    // diagnostics of the options of the last batch call (ttfp_batch_diag)
    std::vector<ttfp_diag> last_batch_diag;
    int last_n_items = 0;
    // tuning (set by ttfp_set_tuning, chosen by the autotuner)
    int tune_maxvol_rounds = 3;           // refinement rounds of maxvol after the block start
    int tune_maxvol_warm = 1;             // maxvol starts from the previous same-direction pivots
    int tune_mm_waves = 8;                // 16-row panels per workgroup of the basis and interpolation products
    int tune_gram_threads = 512;          // threads of a Gram workgroup (two tiles or one tile per wave)
    int tune_mm_panels = 1;               // 16-row panels per wave of the basis and interpolation products
    int tune_interp_bound = 1;            // checking passes skip rows that the row bound clears
    int n_cu = 256;
    int tune_tsqr_lds_kb = 152;
    int tune_graph = 1;                   // graph replay whenever the stream is not the null stream
    int tune_qr = 0;                      // 0: Cholesky QR, passes by the rank threshold; 2 / 3: two / three passes; 1: TSQR
    // the half-sweep flags of the device-side convergence test, read one half sweep behind
    int *h_flags = nullptr;               // pinned host memory, MAX_HALF + 1 ints
    hipEvent_t ev_flag[2] = {nullptr, nullptr};
    // item lists of the half sweeps (launches over the items still active two half sweeps
    // earlier): the device list, and pinned staging for the activity flags read back behind each
    // half sweep and for the lists sent ahead, two of each (list_cap ints apiece)
    int *d_list = nullptr;
    int *h_act = nullptr;
    int *h_list = nullptr;
    size_t list_cap = 0;
    // the items whose pivots moved in a refinement round (length first, list_cap entries after),
    // which the next checking pass takes as its item list; used where the item lists are
    int *d_moved = nullptr;
    bool use_moved = false;
    // allocation-free mode (ttfp_price_batch_noalloc): this device's static scratch array
    char *scratch = nullptr;
    bool noalloc = false;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
    long long prof_launches[TTFP_KERNEL_COUNT] = {0};
    double prof_ms[TTFP_KERNEL_COUNT] = {0};
    double prof_work[TTFP_KERNEL_COUNT] = {0};
};

namespace {

const size_t ALIGN = 256;
constexpr int GRAM_ROWS_HOST = 1024;         // fiber rows per Gram workgroup (k_gram)
constexpr int XF_WAVES_HOST = 12;            // 16-row panels per triangular-transform workgroup (k_xform)
constexpr int LAD_WAVES_HOST = 4;            // 16-point panels per ladder workgroup (k_ladder_core)
constexpr int INNER_RE_HOST = TTFP_MAX_RANK; // row stride of the inner-product environment (k_inner_*)
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ctx->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);        \
            return TTFP_EDEVICE;                                                         \
        }                                                                                \
    } while (0)

struct Launch {
    int BR, G, nlev, maxd, maxrows, maxnc, maxR, maxN;
    double min_rank_eps;       // smallest relative rank threshold of the batch's items
    // Step t of a half sweep (either direction) has at most left[t] = min(R, N^t) row groups of N
    // fiber rows: the index sets grow from one multi-index by at most a factor N per core and
    // never past the rank cap (k_init, k_qrcp). The row-parallel launches of step t are sized by
    // rows[t] = N left[t], not by the buffers' R N rows, so that the first and last cores (N rows)
    // do not launch workgroups that have no rows.
    int left[MAXD], rows[MAXD];
};

// TSQR geometry: leaf blocks of BR = Gl nc rows of the fiber, padded row-major (odd stride
// nc | 1), and merges of G <= 3 triangular factors packed by rows (nc (nc + 1) / 2 entries
// each), both within the LDS budget. Three factors per merge measured fastest at nc = 68 (67.6
// options/s on the d = 5 headline batch of 192 options against 67.0 with four, and 58.2 against 51.3
// at 64 options for four against two unpacked): the merges are bound by the serial chain of
// reflectors, so fewer merges pay, until the longer reflectors cost more than they save.
void tsqr_geometry(int nc, int &BR, int &G, int lds_kb = LDS_BYTES / 1024)
{
    const int cap = std::min(lds_kb * 1024, LDS_BYTES) / (int)sizeof(cplx);
    const int Gl = std::max(2, std::min(cap / (nc * (nc | 1)), 512 / nc));
    BR = Gl * nc;
    G = std::max(2, std::min(cap / (nc * (nc + 1) / 2), 3));
}
size_t tsqr_lds_bytes(int BR, int G, int maxnc)
{
    return std::max((size_t)BR * (maxnc | 1), (size_t)G * maxnc * (maxnc + 1) / 2) * sizeof(cplx);
}
int tsqr_levels(int rows, int BR, int G)
{
    int n = (rows + BR - 1) / BR, l = 1;
    while (n > 1) { n = (n + G - 1) / G; ++l; }
    return l;
}

struct ItemSizes {
    size_t bytes;
    size_t off_m, off_C, off_mJ, off_CJ, off_L, off_a, off_kind, off_I, off_J, off_F, off_Rl, off_Ri, off_perm, off_Y, off_W,
        off_Bt, off_cores, off_M, off_M1, off_M2, off_piv, off_keys, off_Ai, off_Qb, off_Gp, off_Ge, off_Xf, off_Rf;
    int rows_max, nblk_max;
};

ItemSizes item_sizes(int d, int N, int R, int p, int BR)
{
    ItemSizes s;
    const int nc = R + p;
    s.rows_max = R * N;
    s.nblk_max = (s.rows_max + BR - 1) / BR;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    s.off_m = take(sizeof(double) * d);
    s.off_C = take(sizeof(double) * d * d);
    s.off_mJ = take(sizeof(double) * d);
    s.off_CJ = take(sizeof(double) * d * d);
    s.off_L = take(sizeof(double) * d);
    s.off_a = take(sizeof(double) * d);
    s.off_kind = take(sizeof(int) * d);
    s.off_I = take(sizeof(int) * (size_t)(d + 1) * R * d);
    s.off_J = take(sizeof(int) * (size_t)(d + 1) * R * d);
    s.off_F = take(sizeof(cplx) * (size_t)s.rows_max * nc);
    s.off_Rl = take(sizeof(cplx) * 2 * (size_t)s.nblk_max * nc * nc);
    s.off_Ri = take(sizeof(cplx) * (size_t)R * R);
    s.off_perm = take(sizeof(int) * nc);
    s.off_Y = take(sizeof(cplx) * (size_t)s.rows_max * R);
    s.off_W = take(sizeof(cplx) * (size_t)s.rows_max * R);
    s.off_Bt = take(sizeof(cplx) * (size_t)s.rows_max * R);
    s.off_cores = take(sizeof(cplx) * (size_t)d * R * N * R);
    s.off_M = take(sizeof(cplx) * (size_t)d * R * R);
    s.off_M1 = take(sizeof(cplx) * (size_t)d * R * R);
    s.off_M2 = take(sizeof(cplx) * (size_t)d * R * R);
    s.off_piv = take(sizeof(int) * R);
    s.off_keys = take(sizeof(float) * (size_t)s.rows_max * 2);    // keys, then viol
    s.off_Ai = take(sizeof(cplx) * (size_t)R * R);
    const size_t gblk = (size_t)(s.rows_max + GRAM_ROWS_HOST - 1) / GRAM_ROWS_HOST;
    s.off_Qb = take(sizeof(cplx) * (size_t)s.rows_max * nc);
    s.off_Gp = take(sizeof(cplx) * gblk * nc * nc);
    s.off_Ge = take(sizeof(int) * gblk);
    s.off_Xf = take(sizeof(cplx) * (size_t)nc * nc);
    s.off_Rf = take(sizeof(cplx) * (size_t)nc * nc);
    s.bytes = o;
    return s;
}

// The allocation-free entry point's workspace: one static array per GPU, held until the process
// ends. Host code never uses this name as an address: the device address comes from
// hipGetSymbolAddress (once per device, in ttfp_create) and is kept in g_scratch.
static __device__ __align__(256) char scratch[TTFP_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES] = {nullptr};

// Device address of `device`'s scratch array (the device must be current); nullptr on failure.
char *scratch_address(int device, std::string &err)
{
    if (device < 0 || device >= MAX_DEVICES) { err = "device index beyond the scratch table"; return nullptr; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch[device] = (char *)ptr;
    }
    return g_scratch[device];
}

// Device workspace of a chunk: the item arena (bytes), the item array and activity flags
// (n_items) and, in allocation-free mode, the Greeks' moment buffer (moment_elems complex values,
// allocated on first use otherwise). Allocation-free mode carves all of it from the scratch array
// and fails with TTFP_EINVAL when it does not fit.
int ensure_arena(ttfp_ctx *ctx, size_t bytes, size_t n_items, size_t moment_elems)
{
    if (ctx->noalloc) {
        const size_t o_items = 0, o_act = align_up(n_items * sizeof(Item)),
                     o_mom = align_up(o_act + n_items * sizeof(int)), o_arena = align_up(o_mom + moment_elems * sizeof(cplx)),
                     need = o_arena + bytes;
        if (need > (size_t)TTFP_NOALLOC_SCRATCH_BYTES) {
            ctx->last_error = "the batch needs " + std::to_string(need) + " bytes of device workspace; the allocation-free "
                              "entry point has " + std::to_string((size_t)TTFP_NOALLOC_SCRATCH_BYTES);
            return TTFP_EINVAL;
        }
        ctx->d_items = (Item *)(ctx->scratch + o_items);
        ctx->items_cap = n_items;
        ctx->d_active = (int *)(ctx->scratch + o_act);
        ctx->d_moments = (cplx *)(ctx->scratch + o_mom);
        ctx->moments_cap = moment_elems;
        ctx->arena = ctx->scratch + o_arena;
        ctx->arena_bytes = (size_t)TTFP_NOALLOC_SCRATCH_BYTES - o_arena;
        return TTFP_OK;
    }
    if (bytes > ctx->arena_bytes) {
        if (ctx->arena) HIPCHK(hipFree(ctx->arena));
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
        size_t want = std::max(bytes, (size_t)64 << 20);
        if (hipMalloc(&ctx->arena, want) != hipSuccess) {
            ctx->arena = nullptr;
            (void)hipGetLastError();
            ctx->last_error = "device allocation of the workspace failed";
            return TTFP_ENOMEM;
        }
        ctx->arena_bytes = want;
    }
    if (n_items > ctx->items_cap) {
        if (ctx->d_items) HIPCHK(hipFree(ctx->d_items));
        if (ctx->d_active) HIPCHK(hipFree(ctx->d_active));
        size_t cap = std::max(n_items, (size_t)64);
        HIPCHK(hipMalloc(&ctx->d_items, cap * sizeof(Item)));
        HIPCHK(hipMalloc(&ctx->d_active, cap * sizeof(int)));
        ctx->items_cap = cap;
    }
    return TTFP_OK;
}

// Work items of a chunk of options.
struct Batch {
    std::vector<Item> items;
    std::vector<int> item_opt;           // option (within the chunk) of each item
    std::vector<double> item_scale, item_mass;
    std::vector<const TermPlan *> item_term;
    Launch geo;
    // device-side convergence state: per option, per item scale, half-sweep flags (+ counter)
    OptState *d_os = nullptr;
    double *d_scale = nullptr;
    int *d_flags = nullptr;
};

int build_items(ttfp_ctx *ctx, const std::vector<const OptionPlan *> &plans, const std::vector<const ttfp_grid *> &grids,
                Batch &b)
{
    b = Batch();
    int maxnc = 1, maxd = 1, maxrows = 1, maxR = 1, maxN = 2;
    for (size_t o = 0; o < plans.size(); ++o) {
        const ttfp_grid *g = grids[o];
        maxnc = std::max(maxnc, g->max_rank + g->n_enrich);
        maxd = std::max(maxd, plans[o]->d);
        maxrows = std::max(maxrows, g->max_rank * g->N);
        maxR = std::max(maxR, g->max_rank);
        maxN = std::max(maxN, g->N);
    }
    int BR, G;
    tsqr_geometry(maxnc, BR, G, ctx->tune_tsqr_lds_kb);
    double min_eps = 1.0;
    for (size_t o = 0; o < plans.size(); ++o) {
        const ttfp_grid *g = grids[o];
        const double eps = g->rank_tol > 0 ? g->rank_tol : 0.1 * g->tol / std::sqrt((double)std::max(plans[o]->d - 1, 1));
        min_eps = std::min(min_eps, eps);
    }
    b.geo = {BR, G, tsqr_levels(maxrows, BR, G), maxd, maxrows, maxnc, maxR, maxN, min_eps, {}, {}};
    for (int t = 0; t < MAXD; ++t) {
        int left = 0, rows = 0;
        for (size_t o = 0; o < plans.size(); ++o) {
            const ttfp_grid *g = grids[o];
            if (t > plans[o]->d - 2) continue;
            long long l = 1;
            for (int q = 0; q < t && l < g->max_rank; ++q) l *= g->N;
            l = std::min<long long>(l, g->max_rank);
            left = std::max(left, (int)l);
            rows = std::max(rows, (int)l * g->N);
        }
        b.geo.left[t] = std::max(left, 1);
        b.geo.rows[t] = std::max(rows, 1);
    }
    // layout
    std::vector<ItemSizes> sz;
    size_t total = 0;
    for (size_t o = 0; o < plans.size(); ++o) {
        const OptionPlan &P = *plans[o];
        const ttfp_grid *g = grids[o];
        for (size_t t = 0; t < P.terms.size(); ++t) {
            ItemSizes s = item_sizes(P.d, g->N, g->max_rank, g->n_enrich, BR);
            sz.push_back(s);
            total += s.bytes;
        }
    }
    const size_t n_items = sz.size();
    const size_t o_os = total, o_scale = align_up(o_os + plans.size() * sizeof(OptState)),
                 o_flags = align_up(o_scale + n_items * sizeof(double)), aux_end = align_up(o_flags + (MAX_HALF + 1) * sizeof(int));
    int rc = ensure_arena(ctx, aux_end, n_items, n_items * (size_t)(maxd + maxd * maxd));
    if (rc) return rc;
    b.d_os = (OptState *)(ctx->arena + o_os);
    b.d_scale = (double *)(ctx->arena + o_scale);
    b.d_flags = (int *)(ctx->arena + o_flags);
    // fill items and upload the static term data
    std::vector<char> host(0);
    size_t base = 0, idx = 0;
    for (size_t o = 0; o < plans.size(); ++o) {
        const OptionPlan &P = *plans[o];
        const ttfp_grid *g = grids[o];
        for (size_t t = 0; t < P.terms.size(); ++t, ++idx) {
            const TermPlan &tp = P.terms[t];
            const ItemSizes &s = sz[idx];
            char *dev = ctx->arena + base;
            Item it;
            std::memset(&it, 0, sizeof it);
            it.d = P.d;
            it.N = g->N;
            it.R = g->max_rank;
            it.p = g->n_enrich;
            it.opt = (int)o;
            it.term = (int)t;
            it.rank_eps = g->rank_tol > 0 ? g->rank_tol : 0.1 * g->tol / std::sqrt((double)std::max(P.d - 1, 1));
            it.delta = 5e-2;
            {
                const long long per_opt = g->n_err_samples > 0 ? g->n_err_samples : (g->n_err_samples == 0 ? 50000 : 0);
                const long long nt = (long long)P.terms.size();
                it.n_samp = (int)((per_opt + nt - 1) / nt);
            }
            it.seed = g->seed * 0x100000001B3ull + (uint64_t)t * 0x9E3779B97F4A7C15ull + 1;
            it.m = (const double *)(dev + s.off_m);
            it.C = (const double *)(dev + s.off_C);
            it.mJ = (const double *)(dev + s.off_mJ);
            it.CJ = (const double *)(dev + s.off_CJ);
            it.lamT = tp.lamT;
            it.L = (const double *)(dev + s.off_L);
            it.alpha = (const double *)(dev + s.off_a);
            it.kind = (const int *)(dev + s.off_kind);
            it.Iset = (int *)(dev + s.off_I);
            it.Jset = (int *)(dev + s.off_J);
            it.F = (cplx *)(dev + s.off_F);
            it.Rlev = (cplx *)(dev + s.off_Rl);
            it.Rinv = (cplx *)(dev + s.off_Ri);
            it.perm = (int *)(dev + s.off_perm);
            it.Y = (cplx *)(dev + s.off_Y);
            it.W = (cplx *)(dev + s.off_W);
            it.Bt = (cplx *)(dev + s.off_Bt);
            it.cores = (cplx *)(dev + s.off_cores);
            it.M = (cplx *)(dev + s.off_M);
            it.M1 = (cplx *)(dev + s.off_M1);
            it.M2 = (cplx *)(dev + s.off_M2);
            it.piv = (int *)(dev + s.off_piv);
            it.keys = (float *)(dev + s.off_keys);
            it.viol = it.keys + (size_t)s.rows_max;
            it.Ai = (cplx *)(dev + s.off_Ai);
            it.Qb = (cplx *)(dev + s.off_Qb);
            it.Gp = (cplx *)(dev + s.off_Gp);
            it.Ge = (int *)(dev + s.off_Ge);
            it.Xf = (cplx *)(dev + s.off_Xf);
            it.Rf = (cplx *)(dev + s.off_Rf);
            it.rows_max = s.rows_max;
            it.nblk_max = s.nblk_max;
            // static term data: one contiguous host staging block up to off_I
            size_t head = s.off_I;
            if (host.size() < head) host.resize(head);
            std::memset(host.data(), 0, head);
            std::memcpy(host.data() + s.off_m, tp.m.data(), sizeof(double) * P.d);
            std::memcpy(host.data() + s.off_C, tp.C.data(), sizeof(double) * P.d * P.d);
            std::memcpy(host.data() + s.off_mJ, tp.mJ.data(), sizeof(double) * P.d);
            std::memcpy(host.data() + s.off_CJ, tp.CJ.data(), sizeof(double) * P.d * P.d);
            std::memcpy(host.data() + s.off_L, tp.L.data(), sizeof(double) * P.d);
            std::memcpy(host.data() + s.off_a, tp.alpha.data(), sizeof(double) * P.d);
            std::memcpy(host.data() + s.off_kind, tp.kind.data(), sizeof(int) * P.d);
            HIPCHK(hipMemcpyAsync(dev, host.data(), head, hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            b.items.push_back(it);
            b.item_opt.push_back((int)o);
            b.item_scale.push_back(tp.scale);
            b.item_mass.push_back(tp.absmass);
            b.item_term.push_back(&tp);
            base += s.bytes;
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->d_items, b.items.data(), n_items * sizeof(Item), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(b.d_scale, b.item_scale.data(), n_items * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    return TTFP_OK;
}

unsigned cdivu(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// ---- kernel timing: an event pair around each launch of a kernel family
hipEvent_t prof_event(ttfp_ctx *ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
struct ProfScope {
    ttfp_ctx *ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(ttfp_ctx *c, int k) : ctx(c), kind(k)
    {
        if (!ctx->prof) return;
        a = prof_event(ctx);
        b = prof_event(ctx);
        if (a) (void)hipEventRecord(a, ctx->stream);
    }
    ~ProfScope()
    {
        if (!ctx->prof || !a || !b) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->ev_open.push_back({kind, {a, b}});
    }
};
// called after a stream synchronisation: folds the finished event pairs into the totals
void prof_collect(ttfp_ctx *ctx)
{
    for (auto &p : ctx->ev_open) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            ctx->prof_launches[p.first] += 1;
            ctx->prof_ms[p.first] += ms;
        }
        ctx->ev_pool.push_back(p.second.first);
        ctx->ev_pool.push_back(p.second.second);
    }
    ctx->ev_open.clear();
}

// Threads per maxvol workgroup (one workgroup per item): the size that minimises the number of
// rounds of resident workgroups (at most 2048 threads and 160 KiB of LDS per CU, about 15 KiB of
// it static) divided by threads^0.7 (a workgroup's speed grows sublinearly with its size).
// maxvol and its refinement run 1024 threads per workgroup (the Gauss-Jordan inverse holds A in
// the registers of exactly that many threads); rmax^2 complex entries of dynamic LDS.
constexpr unsigned MAXVOL_THREADS = 1024;
// k_maxvol's dynamic LDS holds at least the blocked elimination's panel and trailing parts: 512
// candidate rows x (7 + 1) complex entries (64 KiB)
constexpr int MAXVOL_LDS_MIN = 512 * 8;

// Refinement rounds of maxvol after the block start (TTFP_TUNE_MAXVOL_ROUNDS, default 3): each
// marks the rows of B beyond 1 + delta and swaps them in. More rounds give interpolation nearer to
// dominant, hence crosses that need fewer sweeps and land nearer the exact price: on the d = 5
// headline batch of 192 options (within 1e-6 / options/s), with blocks of the pivots and 192
// violators: 2 rounds 339/576 at 71.3, 3: 380 at 72.2, 4: 412 at 71.9, 6: 400 at 67.3, 10: 406 at
// 67.4; with blocks of up to 448 violators: 3 rounds 413 at 75.5, 4: 404 at 73.1 (one box). A round
// with no violating row costs one early-exit launch.
constexpr int MAXVOL_ROUNDS_MAX = 8;

// Passes of shifted Cholesky QR for a relative rank threshold eps. Each pass resolves the
// singular values above about the square root of its shift (~1e-6 of the largest), relative to
// what the earlier passes left: two passes resolve down to ~1e-12 (with relative errors of 1e-2
// near that floor and below 1e-5 above 1e-10), three down to ~1e-16 (R^H R = F^H F to about the
// shift). TTFP_TUNE_QR 0 takes two passes when every threshold is at least 1e-10, else three.
int cholqr_passes(const ttfp_ctx *ctx, double eps)
{
    if (ctx->tune_qr == 2) return 2;
    if (ctx->tune_qr == 3) return 3;
    return eps >= 1e-10 ? 2 : 3;
}

// Grid order of the row-parallel launches: the fiber, Gram, basis, interpolation and core-sum
// kernels take the item from blockIdx.x and the row block from blockIdx.y, so that every item's
// first row block is dispatched before any item's second. A launch is sized by the step's row
// bound, and the workgroups past an item's actual rows return at once: dispatched between working
// workgroups, such empty ones cost about 0.4 us each (a Gram over 960 items of 3 584 rows took
// 6.1 ms with 16 blocks per item in block-major order and 1.6 ms with its 4 blocks); in this order
// they come at the end of the launch. The transform keeps the block-major order, in which the
// workgroups of one item, which all stage the same Xf, run together (measured faster).

// The fiber's triangular factor by passes of shifted Cholesky QR (k_gram, k_chol, k_xform).
void launch_cholqr(ttfp_ctx *ctx, hipStream_t st, Item *it, ItemList act, int maxrows, unsigned ny, int t, int dir, int npass)
{
    const unsigned gb = cdivu(maxrows, GRAM_ROWS_HOST), gx = cdivu(maxrows, 16 * XF_WAVES_HOST);
    for (int pass = 0; pass < npass; ++pass) {
        if (pass > 0) {
            ProfScope ps(ctx, TTFP_KERNEL_XFORM);
            hipLaunchKernelGGL(k_xform, dim3(gx, ny), dim3(64 * XF_WAVES_HOST), 0, st, it, act, t, dir, pass);
        }
        {
            ProfScope ps(ctx, TTFP_KERNEL_GRAM);
            if (ctx->tune_gram_threads == 1024)
                hipLaunchKernelGGL(k_gram<1024>, dim3(ny, gb), dim3(1024), 0, st, it, act, t, dir, pass);
            else
                hipLaunchKernelGGL(k_gram<512>, dim3(ny, gb), dim3(512), 0, st, it, act, t, dir, pass);
        }
        ProfScope ps(ctx, TTFP_KERNEL_CHOL);
        hipLaunchKernelGGL(k_chol, dim3(ny), dim3(256), 0, st, it, act, t, dir, pass, pass == npass - 1 ? 1 : 0);
    }
}

// The basis and interpolation products with TTFP_TUNE_MM_WAVES waves per workgroup and
// TTFP_TUNE_MM_PANELS 16-row panels per wave.
template <int W, int P>
void launch_basis_t(hipStream_t st, Item *it, ItemList act, long long rows, unsigned ny, int t, int dir)
{
    hipLaunchKernelGGL((k_basis<W, P>), dim3(ny, cdivu(rows, 16 * W * P)), dim3(64 * W), 0, st, it, act, t, dir);
}
void launch_basis(const ttfp_ctx *ctx, hipStream_t st, Item *it, ItemList act, long long rows, unsigned ny, int t, int dir)
{
    const bool w16 = ctx->tune_mm_waves == 16, p2 = ctx->tune_mm_panels == 2;
    if (w16 && p2) launch_basis_t<16, 2>(st, it, act, rows, ny, t, dir);
    else if (w16) launch_basis_t<16, 1>(st, it, act, rows, ny, t, dir);
    else if (p2) launch_basis_t<8, 2>(st, it, act, rows, ny, t, dir);
    else launch_basis_t<8, 1>(st, it, act, rows, ny, t, dir);
}

template <int W, int P>
void launch_interp_t(hipStream_t st, Item *it, ItemList act, long long rows, unsigned ny, int t, int dir, int mode,
                     int bound)
{
    // item-major, except over a list of moved items with a device-side length (block-major: the
    // blocks past its length come last)
    const unsigned nb = cdivu(rows, 16 * W * P);
    hipLaunchKernelGGL((k_interp<W, P>), act.count ? dim3(nb, ny) : dim3(ny, nb), dim3(64 * W), 0, st, it, act, t, dir, mode,
                       bound);
}
void launch_interp(const ttfp_ctx *ctx, hipStream_t st, Item *it, ItemList act, long long rows, unsigned ny, int t, int dir,
                   int mode)
{
    const bool w16 = ctx->tune_mm_waves == 16, p2 = ctx->tune_mm_panels == 2;
    const int b = ctx->tune_interp_bound;
    if (w16 && p2) launch_interp_t<16, 2>(st, it, act, rows, ny, t, dir, mode, b);
    else if (w16) launch_interp_t<16, 1>(st, it, act, rows, ny, t, dir, mode, b);
    else if (p2) launch_interp_t<8, 2>(st, it, act, rows, ny, t, dir, mode, b);
    else launch_interp_t<8, 1>(st, it, act, rows, ny, t, dir, mode, b);
}

// Buffers of the item lists for n items; false (launches over every item) when they cannot be
// allocated.
bool ensure_lists(ttfp_ctx *ctx, size_t n)
{
    if (n <= ctx->list_cap) return true;
    if (ctx->h_act) (void)hipHostFree(ctx->h_act);
    if (ctx->h_list) (void)hipHostFree(ctx->h_list);
    if (ctx->d_list) (void)hipFree(ctx->d_list);
    if (ctx->d_moved) (void)hipFree(ctx->d_moved);
    ctx->h_act = ctx->h_list = ctx->d_list = ctx->d_moved = nullptr;
    ctx->list_cap = 0;
    const size_t cap = std::max(n, (size_t)64);
    if (hipHostMalloc((void **)&ctx->h_act, 2 * cap * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_list, 2 * cap * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&ctx->d_list, cap * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&ctx->d_moved, (cap + 1) * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->h_act) (void)hipHostFree(ctx->h_act);
        if (ctx->h_list) (void)hipHostFree(ctx->h_list);
        if (ctx->d_list) (void)hipFree(ctx->d_list);
        if (ctx->d_moved) (void)hipFree(ctx->d_moved);
        ctx->h_act = ctx->h_list = ctx->d_list = ctx->d_moved = nullptr;
        return false;
    }
    ctx->list_cap = cap;
    return true;
}

int launch_step(ttfp_ctx *ctx, const Launch &g, ItemList act, unsigned ny, int t, int dir, int sweep)
{
    hipStream_t st = ctx->stream;
    Item *it = ctx->d_items;
    {
        ProfScope ps(ctx, TTFP_KERNEL_FIBER);
        hipLaunchKernelGGL(k_fiber, dim3(ny, cdivu((long long)g.left[t] * g.maxnc, 256)), dim3(256), 0, st, it, act, t, dir, 0);
    }
    const int rows = g.rows[t];
    if (ctx->tune_qr != 1) {
        launch_cholqr(ctx, st, it, act, rows, ny, t, dir, cholqr_passes(ctx, g.min_rank_eps));
    } else {
        ProfScope ps(ctx, TTFP_KERNEL_TSQR);
        int n = (rows + g.BR - 1) / g.BR;
        const size_t lds = tsqr_lds_bytes(g.BR, g.G, g.maxnc);
        for (int level = 0; level < g.nlev; ++level) {
            hipLaunchKernelGGL(k_tsqr, dim3((unsigned)std::max(n, 1), ny), dim3(TSQR_THREADS), lds, st, it, act, t, dir, level, g.BR, g.G);
            n = (n + g.G - 1) / g.G;
        }
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_QRCP);
        hipLaunchKernelGGL(k_qrcp, dim3(ny), dim3(QRCP_THREADS), 0, st, it, act, t, dir, ctx->tune_qr != 1 ? 0 : g.BR, g.G);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_BASIS);
        launch_basis(ctx, st, it, act, rows, ny, t, dir);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_MAXVOL);
        const int rm = std::max(g.maxR, 2);
        const size_t lds = (size_t)std::max(rm * rm, MAXVOL_LDS_MIN) * sizeof(cplx);
        hipLaunchKernelGGL(k_maxvol, dim3(ny), dim3(MAXVOL_THREADS), lds, st, it, act, t, dir, rm, ctx->tune_maxvol_warm);
    }
    // checking passes of the interpolation matrix over every row, each followed by a refinement
    // round (both return at once for an item whose rows all satisfy the dominance bound), then the
    // pass that stores B
    // (with the moved-item list, a checking pass after a refinement round runs over the items
    // whose pivots that round moved)
    int *moved = ctx->use_moved ? ctx->d_moved : nullptr;
    for (int round = 0; round < ctx->tune_maxvol_rounds; ++round) {
        {
            ProfScope ps(ctx, TTFP_KERNEL_INTERP);
            const ItemList w = round > 0 && moved ? ItemList(act.active, moved + 1, moved) : act;
            launch_interp(ctx, st, it, w, rows, ny, t, dir, round > 0 ? 1 : 0);
        }
        ProfScope ps(ctx, TTFP_KERNEL_REFINE);
        const int rm = std::max(g.maxR, 2);
        const size_t lds = (size_t)rm * rm * sizeof(cplx);
        if (moved) hipLaunchKernelGGL(k_clear_moved, dim3(1), dim3(64), 0, st, moved);
        hipLaunchKernelGGL(k_maxvol_refine, dim3(ny), dim3(MAXVOL_THREADS), lds, st, it, act, t, dir, rm, moved);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_INTERP);
        launch_interp(ctx, st, it, act, rows, ny, t, dir, 2);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_FINISH);
        hipLaunchKernelGGL(k_finish, dim3(1, ny), dim3(256), 0, st, it, act, t, dir);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_CORESUM);
        hipLaunchKernelGGL(k_core_sum, dim3(ny, cdivu((long long)g.left[t] * g.maxR, 256)), dim3(256), 0, st, it, act, t, dir, 0);
    }
    HIPCHK(hipGetLastError());
    return TTFP_OK;
}

int launch_edge(ttfp_ctx *ctx, const Launch &g, ItemList act, unsigned ny, int dir, int sweep)
{
    hipStream_t st = ctx->stream;
    {
        ProfScope ps(ctx, TTFP_KERNEL_FIBER);
        hipLaunchKernelGGL(k_fiber, dim3(ny, cdivu(g.maxR, 256)), dim3(256), 0, st, ctx->d_items, act, 0, dir, 1);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_CORESUM);
        hipLaunchKernelGGL(k_core_sum, dim3(ny, cdivu((long long)g.maxR * g.maxR, 256)), dim3(256), 0, st, ctx->d_items, act, 0, dir, 1);
    }
    {
        ProfScope ps(ctx, TTFP_KERNEL_CONTRACT);
        hipLaunchKernelGGL(k_contract, dim3(ny), dim3(64), 0, st, ctx->d_items, act);
    }
    HIPCHK(hipGetLastError());
    return TTFP_OK;
}

struct OptResult {
    double price = 0, imag = 0, change = INFINITY, kappa = 0;
    double err_est = NAN;
    long long err_samples = 0;
    int sweeps = 0, capped = 0, converged = 0;
    long long evals = 0, swaps = 0, full_starts = 0;
    int singular = 0;
    double hist[64] = {0};                 // relative change after each half sweep
    int code = TTFP_OK;
};

void fill_diag(const OptResult &r, ttfp_diag *diag)
{
    diag->imag_rel = std::fabs(r.imag) / std::max(std::fabs(r.price), 1e-300);
    diag->kappa = r.kappa;
    diag->last_change = r.change;
    diag->n_evals = r.evals;
    diag->maxvol_swaps = r.swaps;
    diag->maxvol_full_starts = r.full_starts;
    diag->sweeps = r.sweeps;
    diag->rank_capped = r.capped;
    diag->converged = r.converged;
    diag->err_est = r.err_est;
    diag->err_samples = r.err_samples;
}

// Runs TT-cross on every item of the batch until each option's price is stable.
int run_batch(ttfp_ctx *ctx, Batch &b, const std::vector<const ttfp_grid *> &grids, std::vector<OptResult> &res,
              bool greeks, std::vector<std::complex<double>> *moments, int &mstride)
{
    const int n_items = (int)b.items.size();
    const int n_opts = (int)grids.size();
    res.assign(n_opts, OptResult());
    std::vector<int> active(n_items, 1);
    HIPCHK(hipMemcpyAsync(ctx->d_active, active.data(), n_items * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_init, dim3(cdivu(n_items, 64)), dim3(64), 0, ctx->stream, ctx->d_items, n_items);
    HIPCHK(hipGetLastError());
    int max_sweeps = 1;
    for (auto *g : grids) max_sweeps = std::max(max_sweeps, g->max_sweeps);
    const int max_half = std::min(2 * max_sweeps, MAX_HALF);
    // the options' convergence state and the half-sweep flags, on the device
    {
        std::vector<OptState> os(n_opts);
        int first = 0;
        for (int o = 0; o < n_opts; ++o) {
            OptState &st = os[o];
            std::memset(&st, 0, sizeof st);
            st.first = first;
            while (first < n_items && b.item_opt[first] == o) ++first;
            st.count = first - st.first;
            st.max_half = 2 * grids[o]->max_sweeps;
            st.active = 1;
            st.tol = grids[o]->tol;
            st.prev = NAN;
            st.change = INFINITY;
        }
        std::vector<int> flags(MAX_HALF + 1, 0);
        HIPCHK(hipMemcpyAsync(b.d_os, os.data(), n_opts * sizeof(OptState), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(b.d_flags, flags.data(), flags.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));    // the staging vectors go out of scope
    }
    std::vector<Item> host_items(n_items);
    // one half sweep over the items of w (ny of them): the steps of every core, the edge core and
    // the contraction, then the convergence test that switches off the items of finished options
    auto launch_half = [&](ItemList w, unsigned ny, int dir, int sweep) -> int {
        for (int t = 0; ny > 0 && t + 1 < b.geo.maxd; ++t) {
            int rc = launch_step(ctx, b.geo, w, ny, t, dir, sweep);
            if (rc) return rc;
        }
        if (ny > 0) {
            int rc = launch_edge(ctx, b.geo, w, ny, dir, sweep);
            if (rc) return rc;
        }
        hipLaunchKernelGGL(k_converge, dim3(1), dim3(256), 0, ctx->stream, ctx->d_items, ctx->d_active, b.d_os, n_opts, b.d_scale,
                           b.d_flags);
        HIPCHK(hipGetLastError());
        return TTFP_OK;
    };
    // Graph mode: each direction's half sweep is captured once and replayed; the kernels read
    // their shapes, ranks, activity and counters from device memory, so one graph serves every
    // sweep. Capture needs a stream other than the null stream.
    struct Graphs {
        hipGraph_t g[2] = {nullptr, nullptr};
        hipGraphExec_t x[2] = {nullptr, nullptr};
        ~Graphs()
        {
            for (int q = 0; q < 2; ++q) {
                if (x[q]) (void)hipGraphExecDestroy(x[q]);
                if (g[q]) (void)hipGraphDestroy(g[q]);
            }
        }
    } graphs;
    const bool use_graph = ctx->tune_graph && ctx->stream != nullptr && !ctx->noalloc && !ctx->prof;
    const bool compact = !use_graph && !ctx->noalloc && ensure_lists(ctx, (size_t)n_items);
    ctx->use_moved = compact;
    // Half sweeps are queued back to back; after queueing half h the host waits for the flag
    // of half h - 1 (copied into pinned memory behind it), so one half sweep stays queued while
    // the host decides, and the run ends when no option was active after a half sweep.
    for (int h = 0; h < max_half; ++h) {
        const int dir = h & 1, sweep = h >> 1;
        if (use_graph) {
            if (!graphs.x[dir]) {
                HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                int rc = launch_half(ItemList(ctx->d_active), (unsigned)n_items, dir, sweep);
                hipGraph_t gr = nullptr;
                hipError_t e = hipStreamEndCapture(ctx->stream, &gr);
                if (rc) return rc;
                HIPCHK(e);
                graphs.g[dir] = gr;
                HIPCHK(hipGraphInstantiate(&graphs.x[dir], gr, nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(graphs.x[dir], ctx->stream));
        } else {
            ItemList w(ctx->d_active);
            unsigned ny = (unsigned)n_items;
            if (compact && h >= 2) {
                // the items still active after half h - 2, whose flags came back with that half's
                // flag (the host has waited for it); items that finished since return at once
                const int *fl = ctx->h_act + (size_t)(h & 1) * ctx->list_cap;
                int *lst = ctx->h_list + (size_t)(h & 1) * ctx->list_cap;
                ny = 0;
                for (int i = 0; i < n_items; ++i)
                    if (fl[i]) lst[ny++] = i;
                if (ny > 0) HIPCHK(hipMemcpyAsync(ctx->d_list, lst, ny * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
                w = ItemList(ctx->d_active, ctx->d_list);
            }
            int rc = launch_half(w, ny, dir, sweep);
            if (rc) return rc;
        }
        HIPCHK(hipMemcpyAsync(ctx->h_flags + h, b.d_flags + h, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        if (compact)
            HIPCHK(hipMemcpyAsync(ctx->h_act + (size_t)(h & 1) * ctx->list_cap, ctx->d_active, n_items * sizeof(int),
                                  hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipEventRecord(ctx->ev_flag[h & 1], ctx->stream));
        if (h >= 1) {
            HIPCHK(hipEventSynchronize(ctx->ev_flag[(h - 1) & 1]));
            if (!ctx->h_flags[h - 1]) break;
        }
    }
    {
        std::vector<OptState> os(n_opts);
        HIPCHK(hipMemcpyAsync(os.data(), b.d_os, n_opts * sizeof(OptState), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (int o = 0; o < n_opts; ++o) {
            OptResult &r = res[o];
            const OptState &st = os[o];
            r.price = st.price;
            r.imag = st.imag;
            r.change = st.change;
            r.converged = st.converged;
            r.capped = st.capped;
            r.sweeps = st.half;
            for (int q = 0; q < std::min(st.half, 64); ++q) r.hist[q] = st.hist[q];
        }
    }
    // every item takes part in the sampled error estimate and the Greeks
    std::fill(active.begin(), active.end(), 1);
    HIPCHK(hipMemcpyAsync(ctx->d_active, active.data(), n_items * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    bool any_samples = false;
    for (const Item &it : b.items) any_samples |= it.n_samp > 0;
    if (any_samples) {
        ProfScope ps(ctx, TTFP_KERNEL_ERREST);
        hipLaunchKernelGGL(k_err_est, dim3(n_items), dim3(512), 0, ctx->stream, ctx->d_items, ctx->d_active);
        HIPCHK(hipGetLastError());
    }
    if (greeks) {
        mstride = b.geo.maxd + b.geo.maxd * b.geo.maxd;
        size_t need = (size_t)n_items * mstride;
        if (need > ctx->moments_cap) {
            if (ctx->noalloc) { ctx->last_error = "moment buffer beyond the scratch layout"; return TTFP_EINVAL; }
            if (ctx->d_moments) HIPCHK(hipFree(ctx->d_moments));
            HIPCHK(hipMalloc(&ctx->d_moments, need * sizeof(cplx)));
            ctx->moments_cap = need;
        }
        hipLaunchKernelGGL(k_core_moments, dim3(cdivu((long long)b.geo.maxR * b.geo.maxR, 256), b.geo.maxd, n_items), dim3(256), 0,
                           ctx->stream, ctx->d_items, ctx->d_active);
        hipLaunchKernelGGL(k_moments, dim3(n_items), dim3(64), 0, ctx->stream, ctx->d_items, ctx->d_active, ctx->d_moments, mstride);
        HIPCHK(hipGetLastError());
        moments->resize(need);
        HIPCHK(hipMemcpyAsync(moments->data(), ctx->d_moments, need * sizeof(cplx), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(host_items.data(), ctx->d_items, n_items * sizeof(Item), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->prof) prof_collect(ctx);
    {
        // per-option diagnostics from the items, cancellation factor and return code
        std::vector<double> mass(n_opts, 0.0);
        for (int i = 0; i < n_items; ++i) {
            const int o = b.item_opt[i];
            mass[o] += b.item_mass[i];
            res[o].evals += host_items[i].n_evals;
            res[o].swaps += host_items[i].mv_iters;
            res[o].full_starts += host_items[i].mv_full;
            res[o].singular |= host_items[i].mv_singular;
        }
        for (int o = 0; o < n_opts; ++o) {
            OptResult &r = res[o];
            r.kappa = mass[o] / std::max(std::fabs(r.price), 1e-300);
            r.code = (r.converged && !r.capped) ? TTFP_OK : TTFP_ENOTCONV;
            // cancellation beyond the tolerance makes the price meaningless, converged or not
            if (r.kappa * 2.220446049250313e-16 > grids[o]->tol) r.code = TTFP_EPRECISION;
            if (r.singular || !std::isfinite(r.price)) r.code = TTFP_EPRECISION;
        }
    }
    {
        // Sec. IV.B convergence measure over the option's terms, each term's sums weighted by its
        // (positive) quadrature scale
        std::vector<double> ea(n_opts, 0.0), ef(n_opts, 0.0);
        std::vector<long long> ns(n_opts, 0);
        for (int i = 0; i < n_items; ++i) {
            const int o = b.item_opt[i];
            if (host_items[i].n_samp <= 0) continue;
            ea[o] += b.item_scale[i] * host_items[i].err_abs;
            ef[o] += b.item_scale[i] * host_items[i].err_ref;
            ns[o] += host_items[i].n_samp;
        }
        for (int o = 0; o < n_opts; ++o) {
            res[o].err_samples = ns[o];
            res[o].err_est = ns[o] > 0 ? (ef[o] > 0.0 ? ea[o] / ef[o] : (ea[o] > 0.0 ? INFINITY : 0.0)) : NAN;
            // sampled bound on the price's relative error, required when the grid asks for it
            if (grids[o]->certify && res[o].code == TTFP_OK && !(res[o].err_est * res[o].kappa <= grids[o]->tol))
                res[o].code = TTFP_ENOTCONV;
        }
    }
    if (ctx->prof)
        for (const Item &it : host_items)
            for (int q = 0; q < TTFP_KERNEL_COUNT; ++q) ctx->prof_work[q] += it.work[q];
    b.items = host_items;
    return TTFP_OK;
}

// dV/dS0_j and dV/dsigma_j of one option from the node moments of its terms' tensor trains:
// d/dtheta of the integrand is the integrand times -i z.(dm_w) - z^T (dC_w) z / 2, a polynomial
// of degree <= 2 in z, so each Greek is a fixed combination of <TT, z_k> and <TT, z_k z_l>.
void greeks_from_moments(const OptionPlan &P, const Batch &b, const std::vector<std::complex<double>> &mom, int mstride,
                         int first_item, double *delta, double *vega)
{
    const int d = P.d;
    const std::complex<double> I(0.0, 1.0);
    for (int j = 0; j < d; ++j) { delta[j] = 0.0; vega[j] = 0.0; }
    for (size_t t = 0; t < P.terms.size(); ++t) {
        const TermPlan &tp = P.terms[t];
        const std::complex<double> *mu1 = mom.data() + (size_t)(first_item + t) * mstride;
        const std::complex<double> *mu2 = mu1 + d;
        const double sc = tp.scale;
        for (int j = 0; j < d; ++j) {
            std::complex<double> dl = 0.0, vg = 0.0;
            for (int k = 0; k < d; ++k) {
                const double Pkj = tp.P[(size_t)k * d + j];
                dl += (-I * Pkj / P.S0[j]) * mu1[k];
                vg += (I * P.sigma[j] * P.T * Pkj) * mu1[k];
            }
            // quadratic part of the vega weight: -T P_kj sum_b R_jb sigma_b P_lb
            for (int k = 0; k < d; ++k) {
                const double Pkj = tp.P[(size_t)k * d + j];
                if (Pkj == 0.0) continue;
                for (int l = 0; l < d; ++l) {
                    double s = 0.0;
                    for (int bb = 0; bb < d; ++bb) s += P.corr[(size_t)j * d + bb] * P.sigma[bb] * tp.P[(size_t)l * d + bb];
                    vg += (-P.T * Pkj * s) * mu2[(size_t)k * d + l];
                }
            }
            delta[j] += sc * dl.real();
            vega[j] += sc * vg.real();
        }
    }
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *ttfp_strerror(int code)
{
    switch (code) {
    case TTFP_OK: return "ok";
    case TTFP_EINVAL: return "invalid argument";
    case TTFP_ENOMEM: return "device memory exhausted";
    case TTFP_EDEVICE: return "HIP runtime error";
    case TTFP_ENOTCONV: return "tolerance not met (rank cap or sweep limit)";
    case TTFP_EPRECISION: return "precision-limited";
    default: return "unknown error";
    }
}

const char *ttfp_last_error(const ttfp_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

int ttfp_create(ttfp_ctx **out, int device, void *hip_stream)
{
    if (!out) return TTFP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TTFP_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return TTFP_EDEVICE;
    ttfp_ctx *c = new (std::nothrow) ttfp_ctx();
    if (!c) return TTFP_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0) c->n_cu = cus;
    if (hipHostMalloc((void **)&c->h_flags, (MAX_HALF + 1) * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_flag[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_flag[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (c->h_flags) (void)hipHostFree(c->h_flags);
        for (auto e : c->ev_flag)
            if (e) (void)hipEventDestroy(e);
        delete c;
        return TTFP_EDEVICE;
    }
    // the allocation-free entry point's scratch array on this device (its address is looked up
    // once per device; a failure only disables that entry point)
    std::string err;
    c->scratch = scratch_address(device, err);
    if (!c->scratch) c->last_error = err;
    *out = c;
    return TTFP_OK;
}

int ttfp_set_tuning(ttfp_ctx *ctx, int param, int value)
{
    if (!ctx) return TTFP_EINVAL;
    switch (param) {
    case TTFP_TUNE_MAXVOL_ROUNDS:
        if (value < 0 || value > MAXVOL_ROUNDS_MAX) break;
        ctx->tune_maxvol_rounds = value;
        return TTFP_OK;
    case TTFP_TUNE_TSQR_LDS_KB:
        if (value < 16 || value > LDS_BYTES / 1024) break;
        ctx->tune_tsqr_lds_kb = value;
        return TTFP_OK;
    case TTFP_TUNE_GRAPH:
        if (value != 0 && value != 1) break;
        ctx->tune_graph = value;
        return TTFP_OK;
    case TTFP_TUNE_QR:
        if (value < 0 || value > 3) break;
        ctx->tune_qr = value;
        return TTFP_OK;
    case TTFP_TUNE_MAXVOL_WARM:
        if (value != 0 && value != 1) break;
        ctx->tune_maxvol_warm = value;
        return TTFP_OK;
    case TTFP_TUNE_MM_WAVES:
        if (value != 8 && value != 16) break;
        ctx->tune_mm_waves = value;
        return TTFP_OK;
    case TTFP_TUNE_GRAM_THREADS:
        if (value != 512 && value != 1024) break;
        ctx->tune_gram_threads = value;
        return TTFP_OK;
    case TTFP_TUNE_MM_PANELS:
        if (value != 1 && value != 2) break;
        ctx->tune_mm_panels = value;
        return TTFP_OK;
    case TTFP_TUNE_INTERP_BOUND:
        if (value != 0 && value != 1) break;
        ctx->tune_interp_bound = value;
        return TTFP_OK;
    default:
        break;
    }
    ctx->last_error = "bad tuning parameter or value";
    return TTFP_EINVAL;
}

int ttfp_get_tuning(ttfp_ctx *ctx, int param, int *value)
{
    if (!ctx || !value) return TTFP_EINVAL;
    switch (param) {
    case TTFP_TUNE_MAXVOL_ROUNDS: *value = ctx->tune_maxvol_rounds; return TTFP_OK;
    case TTFP_TUNE_TSQR_LDS_KB: *value = ctx->tune_tsqr_lds_kb; return TTFP_OK;
    case TTFP_TUNE_GRAPH: *value = ctx->tune_graph; return TTFP_OK;
    case TTFP_TUNE_QR: *value = ctx->tune_qr; return TTFP_OK;
    case TTFP_TUNE_MAXVOL_WARM: *value = ctx->tune_maxvol_warm; return TTFP_OK;
    case TTFP_TUNE_MM_WAVES: *value = ctx->tune_mm_waves; return TTFP_OK;
    case TTFP_TUNE_GRAM_THREADS: *value = ctx->tune_gram_threads; return TTFP_OK;
    case TTFP_TUNE_MM_PANELS: *value = ctx->tune_mm_panels; return TTFP_OK;
    case TTFP_TUNE_INTERP_BOUND: *value = ctx->tune_interp_bound; return TTFP_OK;
    default: return TTFP_EINVAL;
    }
}

int ttfp_profile_enable(ttfp_ctx *ctx, int enable)
{
    if (!ctx) return TTFP_EINVAL;
    if (!ctx->ev_open.empty()) {
        (void)hipStreamSynchronize(ctx->stream);
        prof_collect(ctx);
    }
    ctx->prof = enable != 0;
    for (int k = 0; k < TTFP_KERNEL_COUNT; ++k) { ctx->prof_launches[k] = 0; ctx->prof_ms[k] = 0.0; ctx->prof_work[k] = 0.0; }
    return TTFP_OK;
}

int ttfp_profile_read(ttfp_ctx *ctx, int kernel, int64_t *launches, double *total_ms, double *work)
{
    if (!ctx || kernel < 0 || kernel >= TTFP_KERNEL_COUNT) return TTFP_EINVAL;
    if (!ctx->ev_open.empty()) {
        (void)hipStreamSynchronize(ctx->stream);
        prof_collect(ctx);
    }
    if (launches) *launches = ctx->prof_launches[kernel];
    if (total_ms) *total_ms = ctx->prof_ms[kernel];
    if (work) *work = ctx->prof_work[kernel];
    return TTFP_OK;
}

int ttfp_destroy(ttfp_ctx *ctx)
{
    if (!ctx) return TTFP_EINVAL;
    (void)hipSetDevice(ctx->device);
    if (!ctx->ev_open.empty()) { (void)hipStreamSynchronize(ctx->stream); prof_collect(ctx); }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto e : ctx->ev_flag)
        if (e) (void)hipEventDestroy(e);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    if (ctx->h_act) (void)hipHostFree(ctx->h_act);
    if (ctx->h_list) (void)hipHostFree(ctx->h_list);
    if (ctx->d_list) (void)hipFree(ctx->d_list);
    if (ctx->d_moved) (void)hipFree(ctx->d_moved);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->d_items) (void)hipFree(ctx->d_items);
    if (ctx->d_active) (void)hipFree(ctx->d_active);
    if (ctx->d_moments) (void)hipFree(ctx->d_moments);
    delete ctx;
    return TTFP_OK;
}

int ttfp_plan(const ttfp_option *opt, const ttfp_grid *grid, int32_t *n_terms, double *L_out, double *alpha_out)
{
    try {
        OptionPlan P;
        std::string err;
        int rc = build_plan(opt, grid, P, err);
        if (rc) return rc;
        if (n_terms) *n_terms = (int32_t)P.terms.size();
        for (size_t t = 0; t < P.terms.size(); ++t)
            for (int k = 0; k < P.d; ++k) {
                if (L_out) L_out[t * P.d + k] = P.terms[t].L[k];
                if (alpha_out) alpha_out[t * P.d + k] = P.terms[t].alpha[k];
            }
        return TTFP_OK;
    } catch (...) {
        return TTFP_EINVAL;
    }
}

}  // extern "C"

namespace {

// The batched pricer behind ttfp_price_batch and ttfp_price_batch_noalloc. With ctx->noalloc the
// whole batch is one chunk whose workspace comes from the scratch array.
int price_batch_impl(ttfp_ctx *ctx, int32_t n, const ttfp_option *opts, const ttfp_grid *grids, double *prices,
                     double *delta, double *vega, int32_t *status)
{
    if (n < 0 || (n > 0 && (!opts || !grids || !prices))) {
        ctx->last_error = "bad batch arguments";
        return TTFP_EINVAL;
    }
    try {
        HIPCHK(hipSetDevice(ctx->device));
        std::vector<OptionPlan> plans(n);
        for (int o = 0; o < n; ++o) {
            std::string err;
            int rc = check_cross_settings(&grids[o], err);
            if (!rc) rc = build_plan(&opts[o], &grids[o], plans[o], err);
            if (rc) {
                ctx->last_error = "option " + std::to_string(o) + ": " + err;
                return rc;
            }
        }
        // chunk options so that one chunk's workspace fits in 70% of the device memory that is
        // free or already held by this context's workspace (at least 4 GiB)
        size_t free_b = 0, total_b = 0;
        if (ctx->noalloc || hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)24 << 30;
        const size_t cap_bytes = ctx->noalloc ? SIZE_MAX
                                              : std::max((size_t)4 << 30, (size_t)(0.7 * (double)(free_b + ctx->arena_bytes)));
        int worst = TTFP_OK;
        ctx->last_batch_diag.assign(n, ttfp_diag());
        size_t greek_off = 0;
        int o0 = 0;
        while (o0 < n) {
            std::vector<const OptionPlan *> cp;
            std::vector<const ttfp_grid *> cg;
            size_t bytes = 0, items = 0;
            int o1 = o0;
            while (o1 < n) {
                const ttfp_grid &g = grids[o1];
                int nc = g.max_rank + g.n_enrich, BR, G;
                tsqr_geometry(std::max(nc, 4), BR, G);
                size_t b1 = item_sizes(plans[o1].d, g.N, g.max_rank, g.n_enrich, std::min(BR, 64)).bytes * plans[o1].terms.size();
                if (o1 > o0 && !ctx->noalloc && (bytes + b1 > cap_bytes || items + plans[o1].terms.size() > 60000)) break;
                bytes += b1;
                items += plans[o1].terms.size();
                cp.push_back(&plans[o1]);
                cg.push_back(&grids[o1]);
                ++o1;
            }
            Batch b;
            int rc = build_items(ctx, cp, cg, b);
            if (rc) return rc;
            std::vector<OptResult> res;
            std::vector<std::complex<double>> mom;
            int mstride = 0;
            const bool want = delta || vega;
            rc = run_batch(ctx, b, cg, res, want, &mom, mstride);
            if (rc) return rc;
            int first_item = 0;
            for (int o = o0; o < o1; ++o) {
                const OptResult &r = res[o - o0];
                fill_diag(r, &ctx->last_batch_diag[o]);
                prices[o] = r.price;
                if (status) status[o] = r.code;
                worst = (r.code < 0 || worst < 0) ? std::min(worst, r.code) : std::max(worst, r.code);
                if (want) {
                    std::vector<double> dl(plans[o].d), vg(plans[o].d);
                    greeks_from_moments(plans[o], b, mom, mstride, first_item, dl.data(), vg.data());
                    for (int j = 0; j < plans[o].d; ++j) {
                        if (delta) delta[greek_off + j] = dl[j];
                        if (vega) vega[greek_off + j] = vg[j];
                    }
                }
                greek_off += plans[o].d;
                first_item += (int)plans[o].terms.size();
            }
            o0 = o1;
        }
        return worst;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return TTFP_EINVAL;
    }
}

// Points a context's workspace at its device's scratch array for one call and restores its own
// buffers afterwards; timing events and graph capture (both allocate) are off meanwhile.
struct NoAllocScope {
    ttfp_ctx *c;
    char *arena;
    size_t arena_bytes, items_cap, moments_cap;
    Item *items;
    int *active;
    cplx *moments;
    bool prof;
    explicit NoAllocScope(ttfp_ctx *ctx)
        : c(ctx), arena(ctx->arena), arena_bytes(ctx->arena_bytes), items_cap(ctx->items_cap),
          moments_cap(ctx->moments_cap), items(ctx->d_items), active(ctx->d_active), moments(ctx->d_moments), prof(ctx->prof)
    {
        c->noalloc = true;
        c->prof = false;
        c->arena = nullptr;
        c->arena_bytes = 0;
        c->d_items = nullptr;
        c->items_cap = 0;
        c->d_active = nullptr;
        c->d_moments = nullptr;
        c->moments_cap = 0;
    }
    ~NoAllocScope()
    {
        c->noalloc = false;
        c->prof = prof;
        c->arena = arena;
        c->arena_bytes = arena_bytes;
        c->d_items = items;
        c->items_cap = items_cap;
        c->d_active = active;
        c->d_moments = moments;
        c->moments_cap = moments_cap;
        // a later ttfp_tt_values / ttfp_tt_export must not read the scratch array
        c->last_items.clear();
        c->last_n_items = 0;
    }
};

}  // namespace

extern "C" {

int ttfp_price_batch(ttfp_ctx *ctx, int32_t n, const ttfp_option *opts, const ttfp_grid *grids, double *prices,
                     double *delta, double *vega, int32_t *status)
{
    if (!ctx) return TTFP_EINVAL;
    return price_batch_impl(ctx, n, opts, grids, prices, delta, vega, status);
}

int ttfp_price_two_trains(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t payoff_rank, double *price,
                          int32_t *ranks_cf, int32_t *ranks_payoff, ttfp_diag *diag)
{
    if (!ctx) return TTFP_EINVAL;
    if (!opt || !grid || !price || payoff_rank < 0 || payoff_rank > TTFP_MAX_RANK) {
        ctx->last_error = "ttfp_price_two_trains: null pointer or payoff_rank outside [0, TTFP_MAX_RANK]";
        return TTFP_EINVAL;
    }
    cplx *dE = nullptr, *dX = nullptr;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        OptionPlan P;
        std::string err;
        int rc = check_cross_settings(grid, err);
        if (!rc) rc = build_plan(opt, grid, P, err);
        if (rc) { ctx->last_error = err; return rc; }
        ttfp_grid gpay = *grid;
        if (payoff_rank > 0) gpay.max_rank = payoff_rank;
        rc = check_cross_settings(&gpay, err);
        if (rc) { ctx->last_error = err; return rc; }
        // the characteristic-function trains (no payoff factors) and the payoff trains (the
        // whole exponent, Gaussian and jump parts, set to zero), on the same per-term grids
        OptionPlan Pcf = P, Ppay = P;
        for (TermPlan &tp : Pcf.terms) tp.kind.assign(P.d, KIND_ONE);
        for (TermPlan &tp : Ppay.terms) {
            std::fill(tp.m.begin(), tp.m.end(), 0.0);
            std::fill(tp.C.begin(), tp.C.end(), 0.0);
            tp.lamT = 0.0;
        }
        std::vector<const OptionPlan *> cp{&Pcf, &Ppay};
        std::vector<const ttfp_grid *> cg{grid, &gpay};
        Batch b;
        rc = build_items(ctx, cp, cg, b);
        if (rc) return rc;
        std::vector<OptResult> res;
        int mstride = 0;
        rc = run_batch(ctx, b, cg, res, false, nullptr, mstride);
        if (rc) return rc;
        const int nt = (int)P.terms.size(), d = P.d;
        HIPCHK(hipMalloc(&dE, sizeof(cplx) * INNER_RE_HOST * INNER_RE_HOST));
        HIPCHK(hipMalloc(&dX, sizeof(cplx) * (size_t)grid->max_rank * grid->N * gpay.max_rank));
        double total = 0.0, imag = 0.0;
        for (int t = 0; t < nt; ++t) {
            const Item &A = b.items[t], &B = b.items[nt + t];
            for (int k = 0; k < d; ++k) {
                const long long nx = (long long)A.crow[k] * A.N * B.ccol[k];
                hipLaunchKernelGGL(k_inner_x, dim3(cdivu(nx, 256)), dim3(256), 0, ctx->stream, ctx->d_items, t, nt + t, k, dE, dX);
                hipLaunchKernelGGL(k_inner_e, dim3(cdivu((long long)B.ccol[k] * A.ccol[k], 256)), dim3(256), 0, ctx->stream,
                                   ctx->d_items, t, nt + t, k, dX, dE);
            }
            HIPCHK(hipGetLastError());
            cplx v;
            HIPCHK(hipMemcpyAsync(&v, dE, sizeof(cplx), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            total += P.terms[t].scale * v.x;
            imag += P.terms[t].scale * v.y;
        }
        (void)hipFree(dE);
        (void)hipFree(dX);
        dE = dX = nullptr;
        *price = total;
        // status: both crosses converged without a rank cap, and the product's cancellation allows
        // the tolerance
        OptResult r = res[0];
        const OptResult &q = res[1];
        r.price = total;
        r.imag = imag;
        r.converged = r.converged && q.converged;
        r.capped = r.capped || q.capped;
        r.sweeps = std::max(r.sweeps, q.sweeps);
        r.evals += q.evals;
        r.swaps += q.swaps;
        r.full_starts += q.full_starts;
        r.singular = r.singular || q.singular;
        r.err_est = std::isnan(r.err_est) ? q.err_est : (std::isnan(q.err_est) ? r.err_est : std::max(r.err_est, q.err_est));
        r.err_samples += q.err_samples;
        double mass = 0.0;
        for (const TermPlan &tp : P.terms) mass += tp.absmass;
        r.kappa = mass / std::max(std::fabs(total), 1e-300);
        r.code = (r.converged && !r.capped) ? TTFP_OK : TTFP_ENOTCONV;
        if (r.kappa * 2.220446049250313e-16 > grid->tol || r.singular || !std::isfinite(total)) r.code = TTFP_EPRECISION;
        for (int t = 0; t < nt; ++t) {
            for (int w = 0; w < 2; ++w) {
                int32_t *rk = w == 0 ? ranks_cf : ranks_payoff;
                if (!rk) continue;
                const Item &it = b.items[w * nt + t];
                rk += (size_t)t * (d + 1);
                rk[0] = 1;
                for (int k = 0; k < d; ++k) rk[k + 1] = it.ccol[k];
            }
        }
        if (diag) fill_diag(r, diag);
        ctx->last_items = b.items;
        ctx->last_n_items = (int)b.items.size();
        return r.code;
    } catch (const std::exception &e) {
        if (dE) (void)hipFree(dE);
        if (dX) (void)hipFree(dX);
        ctx->last_error = e.what();
        return TTFP_EDEVICE;
    }
}

int ttfp_price_ladder(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t n_points,
                      const double *S0_points, const double *K_points, const double *r_points, double *prices,
                      ttfp_diag *diag)
{
    if (!ctx) return TTFP_EINVAL;
    if (!opt || !grid || !prices || !S0_points || !K_points || !r_points || n_points < 1 || n_points > TTFP_MAX_LADDER) {
        ctx->last_error = "ttfp_price_ladder: null pointer or n_points outside [1, TTFP_MAX_LADDER]";
        return TTFP_EINVAL;
    }
    cplx *dW = nullptr, *dT = nullptr, *dV = nullptr;
    double *ddm = nullptr;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        OptionPlan P;
        std::string err;
        int rc = check_cross_settings(grid, err);
        if (!rc) rc = build_plan(opt, grid, P, err);
        if (rc) { ctx->last_error = err; return rc; }
        const int d = P.d, S = n_points, nt = (int)P.terms.size();
        // every point: a valid option with the base's volatilities, correlation, maturity, payoff;
        // its shift of the mean of w per term, and its scale relative to the base's
        std::vector<double> dm((size_t)nt * S * d), ratio(S);
        for (int p = 0; p < S; ++p) {
            ttfp_option o = *opt;
            o.S0 = S0_points + (size_t)p * d;
            o.K = K_points[p];
            o.r = r_points[p];
            OptionPlan Pp;
            rc = build_plan(&o, grid, Pp, err);
            if (rc) { ctx->last_error = "ladder point " + std::to_string(p) + ": " + err; return rc; }
            for (int t = 0; t < nt; ++t)
                for (int k = 0; k < d; ++k) dm[((size_t)t * S + p) * d + k] = Pp.terms[t].m[k] - P.terms[t].m[k];
            ratio[p] = o.K * std::exp(-o.r * o.T) / (opt->K * std::exp(-opt->r * opt->T));
        }
        // the base cross
        std::vector<const OptionPlan *> cp{&P};
        std::vector<const ttfp_grid *> cg{grid};
        Batch b;
        rc = build_items(ctx, cp, cg, b);
        if (rc) return rc;
        std::vector<OptResult> res;
        int mstride = 0;
        rc = run_batch(ctx, b, cg, res, false, nullptr, mstride);
        if (rc) return rc;
        const OptResult &r = res[0];
        // the per-point contractions, term by term and core by core
        int Rmax = 1;
        for (const Item &it : b.items) Rmax = std::max(Rmax, it.R);
        HIPCHK(hipMalloc(&ddm, sizeof(double) * dm.size()));
        HIPCHK(hipMalloc(&dW, sizeof(cplx) * (size_t)S * grid->N));
        HIPCHK(hipMalloc(&dT, sizeof(cplx) * (size_t)S * Rmax * Rmax));
        HIPCHK(hipMalloc(&dV, sizeof(cplx) * (size_t)S * Rmax));
        HIPCHK(hipMemcpyAsync(ddm, dm.data(), sizeof(double) * dm.size(), hipMemcpyHostToDevice, ctx->stream));
        std::vector<double> acc(S, 0.0);
        std::vector<cplx> Pt(S);
        for (int t = 0; t < nt; ++t) {
            const Item &it = b.items[t];
            for (int k = 0; k < d; ++k) {
                hipLaunchKernelGGL(k_ladder_weights, dim3(cdivu((long long)S * it.N, 256)), dim3(256), 0, ctx->stream,
                                   ctx->d_items, t, k, S, ddm + (size_t)t * S * d, dW);
                {
                    ProfScope ps(ctx, TTFP_KERNEL_LADDER);
                    hipLaunchKernelGGL(k_ladder_core, dim3(cdivu(S, 16 * LAD_WAVES_HOST), std::max(it.crow[k], 1)),
                                       dim3(64 * LAD_WAVES_HOST), 0, ctx->stream, ctx->d_items, t, k, S, dW, dT);
                    if (ctx->prof) ctx->prof_work[TTFP_KERNEL_LADDER] += 8.0 * S * (double)it.N * it.crow[k] * it.ccol[k];
                }
                hipLaunchKernelGGL(k_ladder_chain, dim3(S), dim3(64), 0, ctx->stream, ctx->d_items, t, k, S, dT, dV);
            }
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpy2DAsync(Pt.data(), sizeof(cplx), dV, sizeof(cplx) * it.R, sizeof(cplx), S,
                                    hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            for (int p = 0; p < S; ++p) acc[p] += b.item_scale[t] * ratio[p] * Pt[p].x;
        }
        (void)hipFree(ddm);
        (void)hipFree(dW);
        (void)hipFree(dT);
        (void)hipFree(dV);
        ddm = nullptr;
        dW = dT = dV = nullptr;
        for (int p = 0; p < S; ++p) prices[p] = acc[p];
        if (diag) fill_diag(r, diag);
        ctx->last_items = b.items;
        ctx->last_n_items = (int)b.items.size();
        if (ctx->prof) prof_collect(ctx);
        return r.code;
    } catch (const std::exception &e) {
        if (ddm) (void)hipFree(ddm);
        if (dW) (void)hipFree(dW);
        if (dT) (void)hipFree(dT);
        if (dV) (void)hipFree(dV);
        ctx->last_error = e.what();
        return TTFP_EDEVICE;
    }
}

int ttfp_batch_diag(ttfp_ctx *ctx, int32_t i, ttfp_diag *diag)
{
    if (!ctx) return TTFP_EINVAL;
    if (!diag || i < 0 || (size_t)i >= ctx->last_batch_diag.size()) {
        ctx->last_error = "no such option in the last batch";
        return TTFP_EINVAL;
    }
    *diag = ctx->last_batch_diag[i];
    return TTFP_OK;
}

int ttfp_price_batch_noalloc(ttfp_ctx *ctx, int32_t n, const ttfp_option *opts, const ttfp_grid *grids, double *prices,
                             double *delta, double *vega, int32_t *status)
{
    if (!ctx) return TTFP_EINVAL;
    if (!ctx->scratch) {
        ctx->last_error = "the scratch array of this device is unavailable: " + ctx->last_error;
        return TTFP_EDEVICE;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) { ctx->last_error = "hipSetDevice failed"; return TTFP_EDEVICE; }
    NoAllocScope scope(ctx);
    return price_batch_impl(ctx, n, opts, grids, prices, delta, vega, status);
}

int ttfp_price(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, double *price, int32_t *ranks, ttfp_diag *diag)
{
    if (!ctx) return TTFP_EINVAL;
    if (!price) { ctx->last_error = "price is NULL"; return TTFP_EINVAL; }
    try {
        HIPCHK(hipSetDevice(ctx->device));
        OptionPlan P;
        std::string err;
        int rc = check_cross_settings(grid, err);
        if (!rc) rc = build_plan(opt, grid, P, err);
        if (rc) { ctx->last_error = err; return rc; }
        std::vector<const OptionPlan *> cp{&P};
        std::vector<const ttfp_grid *> cg{grid};
        Batch b;
        rc = build_items(ctx, cp, cg, b);
        if (rc) return rc;
        std::vector<OptResult> res;
        int mstride = 0;
        rc = run_batch(ctx, b, cg, res, false, nullptr, mstride);
        if (rc) return rc;
        const OptResult &r = res[0];
        *price = r.price;
        if (ranks) {
            for (size_t t = 0; t < b.items.size(); ++t) {
                const Item &it = b.items[t];
                int32_t *rk = ranks + t * (P.d + 1);
                rk[0] = 1;
                for (int k = 0; k < P.d; ++k) rk[k + 1] = it.ccol[k];
            }
        }
        if (diag) fill_diag(r, diag);
        ctx->last_items = b.items;
        ctx->last_n_items = (int)b.items.size();
        return r.code;
    } catch (const std::exception &e) {
        ctx->last_error = e.what();
        return TTFP_EINVAL;
    }
}

int ttfp_eval_integrand(ttfp_ctx *ctx, const ttfp_option *opt, const ttfp_grid *grid, int32_t term, int64_t npts,
                        const int32_t *idx, double *out)
{
    if (!ctx) return TTFP_EINVAL;
    if (npts < 0 || (npts > 0 && (!idx || !out))) { ctx->last_error = "bad point arguments"; return TTFP_EINVAL; }
    OptionPlan P;
    std::string err;
    int rc = build_plan(opt, grid, P, err);
    if (rc) { ctx->last_error = err; return rc; }
    if (term < 0 || term >= (int)P.terms.size()) { ctx->last_error = "term out of range"; return TTFP_EINVAL; }
    for (int64_t q = 0; q < npts * P.d; ++q)
        if (idx[q] < 0 || idx[q] >= grid->N) { ctx->last_error = "grid index out of range"; return TTFP_EINVAL; }
    if (npts == 0) return TTFP_OK;
    HIPCHK(hipSetDevice(ctx->device));
    const TermPlan &tp = P.terms[term];
    const int d = P.d;
    // one small allocation holding the term data, indices and output
    size_t o_m = 0, o_C = align_up(o_m + 8 * d), o_mJ = align_up(o_C + 8 * d * d), o_CJ = align_up(o_mJ + 8 * d),
           o_L = align_up(o_CJ + 8 * d * d), o_a = align_up(o_L + 8 * d), o_k = align_up(o_a + 8 * d),
           o_i = align_up(o_k + 4 * d), o_o = align_up(o_i + 4 * (size_t)npts * d), total = align_up(o_o + 16 * (size_t)npts);
    char *buf = nullptr;
    Item *dit = nullptr;
    HIPCHK(hipMalloc(&buf, total));
    if (hipMalloc(&dit, sizeof(Item)) != hipSuccess) { (void)hipFree(buf); ctx->last_error = "alloc failed"; return TTFP_ENOMEM; }
    Item it;
    std::memset(&it, 0, sizeof it);
    it.d = d;
    it.N = grid->N;
    it.m = (const double *)(buf + o_m);
    it.C = (const double *)(buf + o_C);
    it.mJ = (const double *)(buf + o_mJ);
    it.CJ = (const double *)(buf + o_CJ);
    it.lamT = tp.lamT;
    it.L = (const double *)(buf + o_L);
    it.alpha = (const double *)(buf + o_a);
    it.kind = (const int *)(buf + o_k);
    hipError_t e = hipSuccess;
    e = e ? e : hipMemcpy(buf + o_m, tp.m.data(), 8 * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_C, tp.C.data(), 8 * d * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_mJ, tp.mJ.data(), 8 * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_CJ, tp.CJ.data(), 8 * d * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_L, tp.L.data(), 8 * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_a, tp.alpha.data(), 8 * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_k, tp.kind.data(), 4 * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(buf + o_i, idx, 4 * (size_t)npts * d, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(dit, &it, sizeof(Item), hipMemcpyHostToDevice);
    if (!e) {
        hipLaunchKernelGGL(k_eval_points, dim3(cdivu(npts, 256)), dim3(256), 0, ctx->stream, dit, (long long)npts,
                           (const int *)(buf + o_i), (cplx *)(buf + o_o));
        e = hipGetLastError();
    }
    e = e ? e : hipStreamSynchronize(ctx->stream);
    e = e ? e : hipMemcpy(out, buf + o_o, 16 * (size_t)npts, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    (void)hipFree(dit);
    if (e) { ctx->last_error = hipGetErrorString(e); return TTFP_EDEVICE; }
    return TTFP_OK;
}

int ttfp_tt_values(ttfp_ctx *ctx, int32_t term, int64_t npts, const int32_t *idx, double *out)
{
    if (!ctx) return TTFP_EINVAL;
    if (ctx->last_n_items == 0) { ctx->last_error = "no tensor train available"; return TTFP_EINVAL; }
    if (term < 0 || term >= ctx->last_n_items) { ctx->last_error = "term out of range"; return TTFP_EINVAL; }
    if (npts <= 0) return npts == 0 ? TTFP_OK : TTFP_EINVAL;
    const Item &h = ctx->last_items[term];
    for (int64_t q = 0; q < npts * h.d; ++q)
        if (idx[q] < 0 || idx[q] >= h.N) { ctx->last_error = "grid index out of range"; return TTFP_EINVAL; }
    HIPCHK(hipSetDevice(ctx->device));
    int *di = nullptr;
    cplx *dout = nullptr;
    HIPCHK(hipMalloc(&di, 4 * (size_t)npts * h.d));
    if (hipMalloc(&dout, 16 * (size_t)npts) != hipSuccess) { (void)hipFree(di); return TTFP_ENOMEM; }
    hipError_t e = hipMemcpy(di, idx, 4 * (size_t)npts * h.d, hipMemcpyHostToDevice);
    if (!e) {
        hipLaunchKernelGGL(k_tt_values, dim3((unsigned)npts), dim3(64), 0, ctx->stream, ctx->d_items, term, (long long)npts, di, dout);
        e = hipGetLastError();
    }
    e = e ? e : hipStreamSynchronize(ctx->stream);
    e = e ? e : hipMemcpy(out, dout, 16 * (size_t)npts, hipMemcpyDeviceToHost);
    (void)hipFree(di);
    (void)hipFree(dout);
    if (e) { ctx->last_error = hipGetErrorString(e); return TTFP_EDEVICE; }
    return TTFP_OK;
}

int ttfp_tt_export(ttfp_ctx *ctx, int32_t term, int32_t *ranks, double *cores, int32_t *set_sizes, int32_t *left,
                   int32_t *right)
{
    if (!ctx) return TTFP_EINVAL;
    if (ctx->last_n_items == 0) { ctx->last_error = "no tensor train available"; return TTFP_EINVAL; }
    if (term < 0 || term >= ctx->last_n_items) { ctx->last_error = "term out of range"; return TTFP_EINVAL; }
    if (!ranks) { ctx->last_error = "ranks is required"; return TTFP_EINVAL; }
    const Item &h = ctx->last_items[term];
    const int d = h.d, N = h.N, R = h.R;
    ranks[0] = 1;
    for (int k = 0; k < d; ++k) ranks[k + 1] = h.ccol[k];
    if (set_sizes)
        for (int k = 0; k <= d; ++k) {
            set_sizes[k] = h.nI[k];
            set_sizes[d + 1 + k] = h.nJ[k];
        }
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (cores) {
        size_t off = 0;
        for (int k = 0; k < d; ++k) {
            const size_t n = (size_t)h.crow[k] * N * h.ccol[k];
            HIPCHK(hipMemcpy(cores + 2 * off, h.cores + (size_t)k * R * N * R, 16 * n, hipMemcpyDeviceToHost));
            off += n;
        }
    }
    if (left) HIPCHK(hipMemcpy(left, h.Iset, sizeof(int) * (size_t)(d + 1) * R * d, hipMemcpyDeviceToHost));
    if (right) HIPCHK(hipMemcpy(right, h.Jset, sizeof(int) * (size_t)(d + 1) * R * d, hipMemcpyDeviceToHost));
    return TTFP_OK;
}

// Raw-matrix entry points: a single item whose shape comes from nI[0] (rows) / nJ[0] (cols).
static int raw_item(ttfp_ctx *ctx, int m, int n, int r, Item &it, char *&buf, int &BR, int &G)
{
    tsqr_geometry(std::max(n, 4), BR, G);
    const int nblk = (m + BR - 1) / BR;
    size_t oF = 0, oRl = align_up(oF + 16 * (size_t)m * n), oY = align_up(oRl + 16 * 2 * (size_t)nblk * n * n),
           oW = align_up(oY + 16 * (size_t)m * r), oBt = align_up(oW + 16 * (size_t)m * r), oP = align_up(oBt + 16 * (size_t)m * r),
           oK = align_up(oP + 4 * (size_t)std::max(r, 1)), oA = align_up(oK + 4 * 2 * (size_t)m),
           gblk = (size_t)(m + GRAM_ROWS_HOST - 1) / GRAM_ROWS_HOST, oQ = align_up(oA + 16 * (size_t)r * r),
           oGp = align_up(oQ + 16 * (size_t)m * n), oGe = align_up(oGp + 16 * gblk * n * n), oXf = align_up(oGe + 4 * gblk),
           oRf = align_up(oXf + 16 * (size_t)n * n), total = align_up(oRf + 16 * (size_t)n * n);
    HIPCHK(hipMalloc(&buf, total));
    std::memset(&it, 0, sizeof it);
    it.d = 1;
    it.N = 1;
    it.R = std::max(r, n);
    it.F = (cplx *)(buf + oF);
    it.Rlev = (cplx *)(buf + oRl);
    it.Y = (cplx *)(buf + oY);
    it.W = (cplx *)(buf + oW);
    it.Bt = (cplx *)(buf + oBt);
    it.piv = (int *)(buf + oP);
    it.keys = (float *)(buf + oK);
    it.viol = it.keys + (size_t)m;
    it.Ai = (cplx *)(buf + oA);
    it.Qb = (cplx *)(buf + oQ);
    it.Gp = (cplx *)(buf + oGp);
    it.Ge = (int *)(buf + oGe);
    it.Xf = (cplx *)(buf + oXf);
    it.Rf = (cplx *)(buf + oRf);
    it.nblk_max = nblk;
    it.rows_max = m;
    it.nI[0] = m;
    it.nJ[0] = n;
    it.rsel = r;
    return TTFP_OK;
}

int ttfp_qr_r(ttfp_ctx *ctx, int32_t m, int32_t n, const double *A, double *R)
{
    if (!ctx) return TTFP_EINVAL;
    if (m < 1 || n < 1 || n > MAXNC || m > TTFP_MAX_RANK * MAXN || !A || !R) { ctx->last_error = "bad qr_r arguments"; return TTFP_EINVAL; }
    HIPCHK(hipSetDevice(ctx->device));
    Item it;
    char *buf = nullptr;
    int BR, G;
    int rc = raw_item(ctx, m, n, 1, it, buf, BR, G);
    if (rc) return rc;
    int *act = nullptr;
    Item *dit = nullptr;
    hipError_t e = hipMalloc(&act, sizeof(int));
    e = e ? e : hipMalloc(&dit, sizeof(Item));
    int one = 1;
    e = e ? e : hipMemcpy(act, &one, sizeof(int), hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(dit, &it, sizeof(Item), hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(it.F, A, 16 * (size_t)m * n, hipMemcpyHostToDevice);
    const cplx *rsrc = it.Rf;
    if (ctx->tune_qr != 1) {
        if (!e) {
            launch_cholqr(ctx, ctx->stream, dit, act, m, 1, 0, 2, ctx->tune_qr == 2 ? 2 : 3);
            e = hipGetLastError();
        }
    } else {
        const int nlev = tsqr_levels(m, BR, G);
        int nb = (m + BR - 1) / BR;
        for (int level = 0; !e && level < nlev; ++level) {
            hipLaunchKernelGGL(k_tsqr, dim3((unsigned)std::max(nb, 1), 1), dim3(TSQR_THREADS), tsqr_lds_bytes(BR, G, std::max(n, 4)),
                               ctx->stream, dit, act, 0, 2, level, BR, G);
            e = hipGetLastError();
            nb = (nb + G - 1) / G;
        }
        // final level
        int cnt = (m + BR - 1) / BR, lf = 0;
        while (cnt > 1) { cnt = (cnt + G - 1) / G; ++lf; }
        rsrc = it.Rlev + (size_t)(lf & 1) * it.nblk_max * n * n;
    }
    e = e ? e : hipStreamSynchronize(ctx->stream);
    e = e ? e : hipMemcpy(R, rsrc, 16 * (size_t)n * n, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    (void)hipFree(act);
    (void)hipFree(dit);
    if (e) { ctx->last_error = hipGetErrorString(e); return TTFP_EDEVICE; }
    return TTFP_OK;
}

int ttfp_maxvol(ttfp_ctx *ctx, int32_t m, int32_t r, const double *A, double delta, int32_t *rows, double *B)
{
    if (!ctx) return TTFP_EINVAL;
    if (m < 1 || r < 1 || r > TTFP_MAX_RANK || r > m || m > TTFP_MAX_RANK * MAXN || !A || !rows || !B || !(delta >= 0)) {
        ctx->last_error = "bad maxvol arguments";
        return TTFP_EINVAL;
    }
    HIPCHK(hipSetDevice(ctx->device));
    Item it;
    char *buf = nullptr;
    int BR, G;
    int rc = raw_item(ctx, m, r, r, it, buf, BR, G);
    if (rc) return rc;
    it.delta = delta;
    int *act = nullptr;
    Item *dit = nullptr;
    hipError_t e = hipMalloc(&act, sizeof(int));
    e = e ? e : hipMalloc(&dit, sizeof(Item));
    int one = 1;
    e = e ? e : hipMemcpy(act, &one, sizeof(int), hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(dit, &it, sizeof(Item), hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(it.Y, A, 16 * (size_t)m * r, hipMemcpyHostToDevice);
    if (!e) {
        const int rm = std::max(r, 2);
        const size_t lds = (size_t)std::max(rm * rm, MAXVOL_LDS_MIN) * sizeof(cplx);
        const unsigned th = MAXVOL_THREADS;
        hipLaunchKernelGGL(k_maxvol, dim3(1), dim3(th), lds, ctx->stream, dit, act, 0, 2, rm, 0);
        // refinement rounds until every row satisfies the dominance bound (each round returns at
        // once when none violates)
        for (int round = 0; round < 8; ++round) {
            launch_interp(ctx, ctx->stream, dit, act, m, 1, 0, 2, round > 0 ? 1 : 0);
            hipLaunchKernelGGL(k_maxvol_refine, dim3(1), dim3(th), lds, ctx->stream, dit, act, 0, 2, rm, (int *)nullptr);
        }
        launch_interp(ctx, ctx->stream, dit, act, m, 1, 0, 2, 2);
        e = hipGetLastError();
    }
    e = e ? e : hipStreamSynchronize(ctx->stream);
    e = e ? e : hipMemcpy(B, it.Bt, 16 * (size_t)m * r, hipMemcpyDeviceToHost);
    e = e ? e : hipMemcpy(rows, it.piv, 4 * (size_t)r, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    (void)hipFree(act);
    (void)hipFree(dit);
    if (e) { ctx->last_error = hipGetErrorString(e); return TTFP_EDEVICE; }
    return TTFP_OK;
}

}  // extern "C"
