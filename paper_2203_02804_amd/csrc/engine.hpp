// Device-side data layout of the batched TT-cross engine.
//
// A work item is one separable term of one option. Every kernel takes the array of
// items and a step index; each workgroup reads its item's shapes from device memory, so
// items of different d, N and rank advance together in one launch, and no host round
// trip is needed between the steps of a half sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ttfp.h"

namespace ttfp {

constexpr int MAXD = TTFP_MAX_D;
constexpr int MAXNC = TTFP_MAX_RANK + 4;     // fiber columns: rank + enrichment
// threads of the column-pivoted QR (one workgroup per item; its LDS allows one per CU)
constexpr int QRCP_THREADS = 1024;
constexpr int MAXN = 1024;                   // nodes per coordinate
constexpr int LDS_BYTES = 152 * 1024;        // per-workgroup LDS budget of the QR kernels
constexpr int TSQR_THREADS = 1024;           // threads of a TSQR workgroup

struct cplx { double x, y; };

struct Item {
    // ---- static description
    int d, N, R, p;            // assets, nodes, rank cap, enrichment columns
    int opt, term;             // owning option and term index
    double rank_eps;           // relative pivot threshold for truncation
    double delta;              // maxvol dominance threshold
    uint64_t seed;
    int n_samp;                // random grid points of the sampled error estimate
    const double *m;           // [d]    mean of w
    const double *C;           // [d*d]  covariance of w
    const double *mJ;          // [d]    Merton jumps: mean of the log-jump sizes in w
    const double *CJ;          // [d*d]  their covariance in w
    double lamT;               // jump rate times maturity (0: no jumps)
    const double *L;           // [d]    half-widths
    const double *alpha;       // [d]    contour shifts
    const int *kind;           // [d]    payoff factor kinds
    // ---- buffers (device)
    int *Iset;                 // [(d+1)][R][d] left multi-indices (coords 0..k-1 used)
    int *Jset;                 // [(d+1)][R][d] right multi-indices (coords k..d-1 used)
    cplx *F;                   // fiber, rows_max x nc_max
    cplx *Rlev;                // two TSQR level buffers, each nblk_max x nc x nc
    cplx *Rinv;                // R x R, inverse of the kept block of the pivoted R
    int *perm;                 // nc, column order of the pivoted QR
    cplx *Y;                   // rows_max x R basis
    cplx *W;                   // rows_max x R maxvol workspace
    cplx *Bt;                  // rows_max x R maxvol output of right-to-left steps
    cplx *cores;               // d slots of R x N x R
    cplx *M;                   // d slots of R x R: core sums over the node index
    cplx *M1, *M2;             // d slots of R x R: first / second node moments (Greeks)
    int *piv;                  // R pivot rows
    cplx *Ai;                  // R x R inverse of the pivot rows of Y (maxvol -> k_interp)
    float *keys;               // rows_max squared row norms of Y (maxvol start)
    float *viol;               // rows_max marks of k_interp: a row's largest |B| above the bound, else 0
    cplx *Qb;                  // rows_max x nc_max: the Cholesky QR's transformed fiber
    cplx *Gp;                  // gram_blocks(rows_max) x nc x nc partial Gram matrices
    int *Ge;                   // gram_blocks(rows_max) power-of-two exponents of the partials
    cplx *Xf;                  // nc x nc inverse of the last Cholesky factor
    cplx *Rf;                  // nc x nc running triangular factor (the fiber's R after the last pass)
    int rows_max, nblk_max;
    // ---- dynamic state
    int nI[MAXD + 1], nJ[MAXD + 1];   // sizes of the left / right index sets
    int crow[MAXD], ccol[MAXD];       // core shapes
    int rsel;                         // rank selected in the current step
    int gram_e;                       // exponent of the power-of-two scaling of the fiber's Gram
    int half;                         // half sweeps completed (counter of the random draws)
    int capped;
    long long n_evals;
    long long mv_iters;               // maxvol swaps performed (diagnostic)
    long long mv_full;                // maxvol starts taken over all rows (degenerate candidate block)
    int mv_singular;                  // a maxvol start matrix was exactly singular
    int mv_viol;                      // k_interp found rows with |B_ij| > 1 + delta
    int mv_dirty;                     // the pivots moved since B was last formed
    double mv_colmax;                 // largest squared column norm of A^{-1} (the checking passes' row bound)
    double work[TTFP_KERNEL_COUNT];   // algorithmic work per kernel family (bytes or flops)
    cplx P;                           // latest contraction of the tensor train
    double err_abs, err_ref;          // sampled error: sum |TT - A| and sum |A| over n_samp points
};

// Convergence state of one option, kept on the device so that the host does not read the items
// between half sweeps (k_converge updates it after every half sweep).
constexpr int MAX_HALF = 128;                 // half sweeps (max_sweeps <= 64)
struct OptState {
    int first, count;                 // the option's items (contiguous)
    int max_half;                     // 2 max_sweeps
    int active, converged, capped, half;
    double tol;
    double prev;                      // price after the previous half sweep (NaN before the first)
    double price, imag, change;       // latest contraction and relative change
    double hist[64];                  // relative change after each half sweep
};

// The items a launch works on: block b of the launch's item dimension takes item list[b], or item
// b when the launch has no list; an item whose activity flag is 0 returns at once. The half sweeps
// launch over the items that were still active a little earlier (the flags only ever turn off), so
// that finished options cost no workgroups.
// A list may also carry a device-side length (count): block b >= *count then has no item (-1).
struct ItemList {
    const int *active;
    const int *list;
    const int *count;
    __host__ __device__ ItemList(const int *a, const int *l = nullptr, const int *n = nullptr) : active(a), list(l), count(n) {}
    __device__ int item(int b) const { return list ? (count && b >= *count ? -1 : list[b]) : b; }
};

// Step addressing: dir 0 = left-to-right (core k = t), dir 1 = right-to-left (core k = d-1-t).
__host__ __device__ inline int step_core(const Item &it, int t, int dir) { return dir == 0 ? t : it.d - 1 - t; }

}  // namespace ttfp
