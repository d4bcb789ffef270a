// HIP kernels of the TT-cross pricer (gfx950, wave64).
//
// One half sweep of TT-cross (Sec. IV.B) is, for every core k in order:
//   k_fiber    evaluate the fiber A[I_k, i, J_{k+1}] (+ random enrichment columns)   (complex FP64)
//   k_tsqr     triangular factor of a QR of the fiber, TSQR over LDS-resident row blocks
//   k_qrcp     column-pivoted QR of that factor: rank by pivot size, inverse of the kept block
//   k_basis    orthonormal basis of the kept fiber columns
//   k_maxvol   rows of a dominant submatrix (maxvol); k_interp the interpolating core B
//   k_finish   next index set and core shape
//   k_core_sum core summed over the node index (the quadrature weights are uniform)
// then k_fiber on the edge core and k_contract (Sec. IV.A inner product with the weights).
#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace ttfp {

// ------------------------------------------------------------------ complex helpers
// Global memory through its own address space. The items hold generic pointers, and loads and
// stores through generic pointers compile to flat instructions, which count against the same wait
// counter as LDS accesses: a loop that waits for its LDS operands would also wait for every global
// load it issued ahead of time. The hot loops load and store through these instead.
#define GLOBAL_AS __attribute__((address_space(1)))
typedef double gdbl2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx gld(const cplx *p)
{
    const gdbl2_t v = *(const GLOBAL_AS gdbl2_t *)p;
    return {v.x, v.y};
}
__device__ __forceinline__ float gld(const float *p) { return *(const GLOBAL_AS float *)p; }
__device__ __forceinline__ void gst(cplx *p, cplx v) { *(GLOBAL_AS gdbl2_t *)p = gdbl2_t{v.x, v.y}; }
__device__ __forceinline__ void gst(float *p, float v) { *(GLOBAL_AS float *)p = v; }

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) * b
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b)
{
    // scaled division (Smith)
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, den = b.x + b.y * r;
        return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
    }
    double r = b.x / b.y, den = b.x * r + b.y;
    return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
__device__ __forceinline__ cplx cexp_(cplx a)
{
    double e = exp(a.x), s, c;
    sincos(a.y, &s, &c);
    return {e * c, e * s};
}


// Cross-lane moves by DPP (row-local permutations that run at VALU speed, unlike the LDS-routed
// ds_bpermute of a generic shuffle). CTRL: 0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm
// [2,3,0,1] (lane ^ 2), 0x141 row_half_mirror (lane 7 - i within 8), 0x140 row_mirror (lane
// 15 - i within 16). After the four steps every lane of a row of 16 holds the row's sum.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double read_lane(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Row exchanges of gfx950 (v_permlane16_swap / v_permlane32_swap on two copies of v): every lane
// gets the values of rows {2q, 2q+1} (16-lane rows, swap16) or of halves {0, 1} (32-lane halves,
// swap32) that hold it, lower one in lo, upper one in hi, in the same order in every lane.
__device__ __forceinline__ void swap16(double v, double &lo, double &hi)
{
    const long long b = __double_as_longlong(v);
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    lo = __longlong_as_double(((long long)h[0] << 32) | l[0]);
    hi = __longlong_as_double(((long long)h[1] << 32) | l[1]);
}
__device__ __forceinline__ void swap32(double v, double &lo, double &hi)
{
    const long long b = __double_as_longlong(v);
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    lo = __longlong_as_double(((long long)h[0] << 32) | l[0]);
    hi = __longlong_as_double(((long long)h[1] << 32) | l[1]);
}
// sum over each group of S adjacent lanes (S = 1, 2, 4, 8, 16), left in every lane of the group
__device__ __forceinline__ double seg_sum(double v, int S)
{
    if (S >= 2) v += dpp_move<0xB1>(v);
    if (S >= 4) v += dpp_move<0x4E>(v);
    if (S >= 8) v += dpp_move<0x141>(v);
    if (S >= 16) v += dpp_move<0x140>(v);
    return v;
}
// largest value over each group of S adjacent lanes (S = 1, 2, 4, 8, 16), in every lane of it
__device__ __forceinline__ double seg_max(double v, int S)
{
    if (S >= 2) v = fmax(v, dpp_move<0xB1>(v));
    if (S >= 4) v = fmax(v, dpp_move<0x4E>(v));
    if (S >= 8) v = fmax(v, dpp_move<0x141>(v));
    if (S >= 16) v = fmax(v, dpp_move<0x140>(v));
    return v;
}
// sum / max over the 64 lanes of a wave (all lanes active), returned in every lane as
// (row0 + row1) + (row2 + row3), bit-identical across lanes
__device__ __forceinline__ double wave_sum(double v)
{
    double lo, hi;
    v = seg_sum(v, 16);
    swap16(v, lo, hi);
    swap32(lo + hi, lo, hi);
    return lo + hi;
}
// NV = 2, 4 or 8 sums over the 64 lanes of a wave at once, left in v (the same in every lane).
// Exchange steps halve the values a lane carries (partner lane ^ 1, lane ^ 2, then row_ror:4,
// which keeps bits 0 and 1 of the lane and flips bit 2), plain steps over the lane bits left
// (lane ^ 2, row_ror:4, row_ror:8) finish each 16-lane row, the row swaps cross the wave, and
// one readlane per value broadcasts it (value k ends in the lanes whose low log2(NV) bits are k
// reversed). For eight values this is about half the instructions of eight wave_sums.
template <int NV>
__device__ __forceinline__ void wave_sum_n(double (&v)[NV])
{
    static_assert(NV == 2 || NV == 4 || NV == 8, "2, 4 or 8 values");
    const int lane = threadIdx.x & 63;
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    double x;
    if constexpr (NV == 8) {
        double u[4], w[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double send = b0 ? v[k] : v[k + 4], keep = b0 ? v[k + 4] : v[k];
            u[k] = keep + dpp_move<0xB1>(send);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double send = b1 ? u[k] : u[k + 2], keep = b1 ? u[k + 2] : u[k];
            w[k] = keep + dpp_move<0x4E>(send);
        }
        const double send = b2 ? w[0] : w[1], keep = b2 ? w[1] : w[0];
        x = keep + dpp_move<0x124>(send);
    } else if constexpr (NV == 4) {
        double u[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double send = b0 ? v[k] : v[k + 2], keep = b0 ? v[k + 2] : v[k];
            u[k] = keep + dpp_move<0xB1>(send);
        }
        const double send = b1 ? u[0] : u[1], keep = b1 ? u[1] : u[0];
        x = keep + dpp_move<0x4E>(send);
        x += dpp_move<0x124>(x);
    } else {
        const double send = b0 ? v[0] : v[1], keep = b0 ? v[1] : v[0];
        x = keep + dpp_move<0xB1>(send);
        x += dpp_move<0x4E>(x);
        x += dpp_move<0x124>(x);
    }
    x += dpp_move<0x128>(x);
    double lo, hi;
    swap16(x, lo, hi);
    swap32(lo + hi, lo, hi);
    x = lo + hi;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        // lane holding value k: k's low bits reversed
        const int l = NV == 8 ? ((k & 1) << 2 | (k & 2) | (k >> 2)) : NV == 4 ? ((k & 1) << 1 | (k >> 1)) : k;
        v[k] = read_lane(x, l);
    }
}
__device__ __forceinline__ double wave_max(double v)
{
    double lo, hi;
    v = fmax(v, dpp_move<0xB1>(v));
    v = fmax(v, dpp_move<0x4E>(v));
    v = fmax(v, dpp_move<0x141>(v));
    v = fmax(v, dpp_move<0x140>(v));
    swap16(v, lo, hi);
    swap32(fmax(lo, hi), lo, hi);
    return fmax(lo, hi);
}

// Scalars of a Householder reflector. The column is scaled by s = 2^-e, a power of two (e = 0 for
// a column that needs no scaling, else the one that takes its largest magnitude into [0.5, 1):
// exact, and cheaper than a division); sqs is the sum of squared moduli of the scaled entries
// below the leading one, x0 the unscaled leading entry. Returns the factor cf that turns an
// unscaled entry below the leading one into w_i, alpha = -phase(x0) |x| and
// tau = (|x0| + |x|) / |x| (in [1, 2]).
struct ReflScalars {
    cplx cf, alpha;
    double tau;
};
__device__ __forceinline__ ReflScalars reflector_scalars(cplx x0, double s, int e, double sqs)
{
    const cplx x0s = {x0.x * s, x0.y * s};
    // |x_j|: squares below 1e-300 keep only a few digits, and a phase formed from them is
    // not of unit modulus (the reflector would not be unitary); hypot then
    double a0 = sqrt(x0s.x * x0s.x + x0s.y * x0s.y);
    if (a0 < 1e-150) a0 = hypot(x0s.x, x0s.y);
    const double nrm = sqrt(sqs + a0 * a0);
    const double ra = a0 > 1e-300 ? 1.0 / a0 : 0.0;
    const cplx ph = a0 > 1e-300 ? cplx{x0s.x * ra, x0s.y * ra} : cplx{1.0, 0.0};
    // w_i = x_i / v_j with v_j = phase (|x_j| + |x|) (in units of 2^e)
    const double den = 1.0 / (a0 + nrm);
    ReflScalars r;
    r.cf = {ph.x * den * s, -ph.y * den * s};
    r.alpha = {-ldexp(ph.x * nrm, e), -ldexp(ph.y * nrm, e)};
    r.tau = (a0 + nrm) / nrm;
    return r;
}

struct ArgMax { double v; int i; };

__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b)
{
    if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
    return a;
}

// argmax within a wave (ties: lowest index) by DPP row permutations and readlanes: better() is a
// total order on (value, index), so the mirror steps leave every lane of a row with the row's best
template <int CTRL>
__device__ __forceinline__ ArgMax dpp_best(ArgMax a)
{
    ArgMax b;
    b.v = dpp_move<CTRL>(a.v);
    b.i = __builtin_amdgcn_update_dpp(0, a.i, CTRL, 0xF, 0xF, false);
    return better(a, b);
}
// best (value, lowest index) over the 64 lanes of a wave, in every lane
__device__ __forceinline__ ArgMax wave_argmax(ArgMax a)
{
    a = dpp_best<0xB1>(a);
    a = dpp_best<0x4E>(a);
    a = dpp_best<0x141>(a);
    a = dpp_best<0x140>(a);
    for (int l = 16; l < 64; l += 16) a = better(a, ArgMax{read_lane(a.v, l), __builtin_amdgcn_readlane(a.i, l)});
    return better(ArgMax{read_lane(a.v, 0), __builtin_amdgcn_readlane(a.i, 0)}, a);
}
// Householder reflector for the column x = (x_j, ..., x_{n-1}) (entry i at x[i * stride]), made by
// wave 0 of the workgroup. The reflector is H = I - tau w w^H with w_j = 1, chosen so that
// H x = (alpha, 0, ..., 0) with alpha = -phase(x_j) |x|. Every quantity is formed from the column
// scaled by the power of two that takes its largest entry into [0.5, 1), so columns of any
// magnitude (integrand values span hundreds of decades) neither underflow to a spurious zero norm
// nor overflow the reflector (tau lies in [1, 2]); a column below 1e-280 in magnitude is left as
// it is (tau = 0). On return x holds w
// (x_j = 1) and the wave's lane 0 has written alpha to *alpha_out and tau to *tau_out.
__device__ void make_reflector(cplx *x, int stride, int j, int n, cplx *alpha_out, double *tau_out)
{
    const int lane = threadIdx.x & 63;
    double mx = 0.0;
    for (int i = j + lane; i < n; i += 64) mx = fmax(mx, fmax(fabs(x[(size_t)i * stride].x), fabs(x[(size_t)i * stride].y)));
    mx = wave_max(mx);
    if (!(mx >= 1e-280) || !(mx <= 1e300)) {
        if (lane == 0) {
            *alpha_out = x[(size_t)j * stride];
            *tau_out = 0.0;
        }
        return;
    }
    int e;
    frexp(mx, &e);
    const double sc = ldexp(1.0, -e);
    double sq = 0.0;
    for (int i = j + 1 + lane; i < n; i += 64) {
        const cplx v = x[(size_t)i * stride];
        sq += cabs2(cplx{v.x * sc, v.y * sc});
    }
    sq = wave_sum(sq);
    const ReflScalars r = reflector_scalars(x[(size_t)j * stride], sc, e, sq);
    for (int i = j + 1 + lane; i < n; i += 64) x[(size_t)i * stride] = cmul(x[(size_t)i * stride], r.cf);
    if (lane == 0) {
        x[(size_t)j * stride] = {1.0, 0.0};
        *alpha_out = r.alpha;
        *tau_out = r.tau;
    }
}

// ------------------------------------------------------------------ counter-based generator
// SplitMix64 finaliser (Steele, Lea and Flood, 2014) applied to a counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ int rand_index(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, int n)
{
    uint64_t h = splitmix64(splitmix64(splitmix64(seed ^ a) ^ b) ^ c);
    return (int)(((h >> 32) * (uint64_t)n) >> 32);
}

// ------------------------------------------------------------------ integrand (one entry)
// exp(-i z.m - z^T C z / 2) * prod_k h_k(z_k),  z_k = -L_k + (i_k + 1/2) 2L_k/N + i alpha_k:
// the Gaussian characteristic function at -z (Sec. III.C) times the payoff factor transforms.
// Kinds: 0 call/put factor 1/(iz(1+iz)); 1 indicator w < 0, 1/(iz); 2 indicator w > 0, -1/(iz);
// 3 coordinate of the single-strip call on the minimum, 1/(iz), whose term also carries the
// joint factor (-1)^(d+1) / (1 + i sum_k z_k) (strip_joint).
__device__ __forceinline__ cplx factor(int kind, cplx z)
{
    if (kind == 4) return {1.0, 0.0};             // no payoff factor
    cplx iz = {-z.y, z.x};
    if (kind == 0) return cdiv({1.0, 0.0}, cmul(iz, {1.0 + iz.x, iz.y}));
    cplx v = cdiv({1.0, 0.0}, iz);
    return kind == 2 ? cplx{-v.x, -v.y} : v;
}
// (-1)^(d+1) / (1 + i s), s = sum_k z_k
__device__ __forceinline__ cplx strip_joint(int d, cplx s)
{
    return cdiv({(d & 1) ? 1.0 : -1.0, 0.0}, {1.0 - s.y, s.x});
}

__device__ cplx integrand(const Item &it, const int *idx)
{
    const int d = it.d;
    const double invN = 1.0 / it.N;
    cplx z[MAXD];
    for (int k = 0; k < d; ++k) {
        double L = it.L[k];
        z[k] = {-L + (idx[k] + 0.5) * 2.0 * L * invN, it.alpha[k]};
    }
    cplx e = {0.0, 0.0}, h = {1.0, 0.0}, zs = {0.0, 0.0}, ej = {0.0, 0.0};
    for (int k = 0; k < d; ++k) {
        const double *Ck = it.C + k * d;
        cplx q = {0.0, 0.0};
        for (int l = 0; l < d; ++l) q = {q.x + Ck[l] * z[l].x, q.y + Ck[l] * z[l].y};
        // z_k * (-i m_k - q/2)
        cplx w = {-0.5 * q.x, -it.m[k] - 0.5 * q.y};
        e = cadd(e, cmul(z[k], w));
        if (it.lamT > 0.0) {
            const double *CJk = it.CJ + k * d;
            cplx qj = {0.0, 0.0};
            for (int l = 0; l < d; ++l) qj = {qj.x + CJk[l] * z[l].x, qj.y + CJk[l] * z[l].y};
            ej = cadd(ej, cmul(z[k], {-0.5 * qj.x, -it.mJ[k] - 0.5 * qj.y}));
        }
        h = cmul(h, factor(it.kind[k], z[k]));
        zs = cadd(zs, z[k]);
    }
    if (it.lamT > 0.0) {
        // Merton jumps: exp(lamT (exp(-i z.mJ - z^T CJ z / 2) - 1))
        const cplx g = cexp_(ej);
        e = cadd(e, {it.lamT * (g.x - 1.0), it.lamT * g.y});
    }
    if (it.kind[0] == 3) h = cmul(h, strip_joint(d, zs));
    return cmul(cexp_(e), h);
}

// ------------------------------------------------------------------ shapes of a step
struct StepShape {
    int k, rows, ncb, nc;   // core, fiber rows, base columns, columns incl. enrichment
    bool valid;
};

// mode 0: interior step t of direction dir; mode 1: edge core of that direction;
// dir 2: raw matrix entry points (rows / columns stored in rsel / nI[0]).
__device__ __forceinline__ StepShape step_shape(const Item &it, int t, int dir, int mode)
{
    StepShape s;
    s.valid = true;
    const int d = it.d;
    if (dir == 2) {
        s.k = 0;
        s.rows = it.nI[0];
        s.ncb = s.nc = it.nJ[0];
        return s;
    }
    if (mode == 0) {
        if (t > d - 2) { s.valid = false; return s; }
        s.k = step_core(it, t, dir);
    } else {
        s.k = dir == 0 ? d - 1 : 0;
    }
    const int p = mode == 0 ? it.p : 0;
    if (dir == 0) {
        s.rows = it.nI[s.k] * it.N;
        s.ncb = it.nJ[s.k + 1];
    } else {
        s.rows = it.N * it.nJ[s.k + 1];
        s.ncb = it.nI[s.k];
    }
    s.nc = s.ncb + p;
    return s;
}

// ------------------------------------------------------------------ init
__global__ void k_init(Item *items, int n_items)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_items) return;
    Item &it = items[j];
    const int d = it.d, N = it.N, R = it.R;
    it.nI[0] = 1;
    it.nJ[d] = 1;
    it.n_evals = 0;
    it.half = 0;
    it.mv_iters = 0;
    it.mv_full = 0;
    it.mv_singular = 0;
    it.mv_viol = 0;
    it.mv_dirty = 0;
    it.mv_colmax = INFINITY;
    for (int q = 0; q < TTFP_KERNEL_COUNT; ++q) it.work[q] = 0.0;
    it.capped = 0;
    long long cnt = 1;
    for (int k = d - 1; k >= 1; --k) {
        cnt = cnt * N;
        if (cnt > R) cnt = R;
        int nj = (int)cnt;
        it.nJ[k] = nj;
        int *Jk = it.Jset + (size_t)k * R * d;
        const int *Jk1 = it.Jset + (size_t)(k + 1) * R * d;
        for (int b = 0; b < nj; ++b) {
            int lo = N >= 4 ? N / 4 : 0, span = N >= 4 ? N / 2 : N;
            Jk[b * d + k] = lo + rand_index(it.seed, 1, (uint64_t)k, (uint64_t)b, span);
            if (k + 1 < d) {
                int bp = rand_index(it.seed, 2, (uint64_t)k, (uint64_t)b, it.nJ[k + 1]);
                for (int c = k + 1; c < d; ++c) Jk[b * d + c] = Jk1[bp * d + c];
            }
        }
    }
}

// ------------------------------------------------------------------ fiber evaluation
// One thread per (row group g, column c) pair, looping over the node index i of core k.
// Left-to-right: g = left index a, c = right index b, row = a N + i.
// Right-to-left: g = right index b, c = left index a, row = i nb + b.
// Everything that does not depend on i is formed once per pair:
//   E_0 = sum_{l != k} z_l (-i m_l) - 1/2 sum_{l,l' != k} z_l C_ll' z_l',
//   tau = -sum_{l != k} C_kl z_l,   H = prod_{l != k} h_l(z_l),
// so that each entry costs one complex multiply-add, one exp and one sincos:
//   F = exp(E_0 + z_k tau + c_k(i)) H h_k(z_k),  c_k(i) = z_k (-i m_k) - C_kk z_k^2 / 2,
// with c_k and h_k tabulated per node in LDS. With Merton jumps the exponent gains
// lamT (exp(J_0 + z_k tau_J + j_k(i)) - 1), J_0, tau_J and j_k formed from mJ and CJ the same way:
// one more exp and sincos per entry.
__global__ __launch_bounds__(256) void k_fiber(Item *items, ItemList work, int t, int dir, int mode)
{
    __shared__ cplx ctab[MAXN];
    __shared__ cplx htab[MAXN];
    __shared__ cplx jtab[MAXN];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, mode);
    if (!s.valid) return;
    const int d = it.d, N = it.N, R = it.R, k = s.k;
    const int ng = (dir == 0) ? s.rows / N : it.nJ[k + 1];     // row groups
    const long long pairs = (long long)ng * s.nc;
    if ((long long)blockIdx.y * blockDim.x >= pairs) return;
    const long long total = (long long)s.rows * s.nc;
    if (blockIdx.y == 0 && threadIdx.x == 0) {
        if (mode == 1) {
            if (dir == 0) { it.crow[k] = it.nI[k]; it.ccol[k] = 1; }
            else { it.crow[k] = 1; it.ccol[k] = it.nJ[1]; }
            it.n_evals += total;
        }
        it.work[TTFP_KERNEL_FIBER] += 16.0 * (double)total;
    }
    // node tables of coordinate k
    const double Lk = it.L[k], etak = 2.0 * Lk / N, ak = it.alpha[k], mk = it.m[k], Ckk = it.C[k * d + k];
    const int kindk = it.kind[k];
    const bool jumps = it.lamT > 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const cplx z = {-Lk + (i + 0.5) * etak, ak};
        const cplx w = {-0.5 * Ckk * z.x, -mk - 0.5 * Ckk * z.y};     // -i m_k - C_kk z / 2
        ctab[i] = cmul(z, w);
        htab[i] = factor(kindk, z);
        if (jumps) {
            const double CJkk = it.CJ[k * d + k];
            jtab[i] = cmul(z, {-0.5 * CJkk * z.x, -it.mJ[k] - 0.5 * CJkk * z.y});
        }
    }
    __syncthreads();
    const long long pidx = (long long)blockIdx.y * blockDim.x + threadIdx.x;
    if (pidx >= pairs) return;
    const int g = (int)(pidx / s.nc), c = (int)(pidx % s.nc);
    const int a = (dir == 0) ? g : c;          // left multi-index
    const int b = (dir == 0) ? c : g;          // right multi-index
    const uint64_t ctr = ((uint64_t)it.half << 40) ^ ((uint64_t)dir << 32) ^ ((uint64_t)t << 16);
    // nodes of every coordinate but k
    cplx z[MAXD];
    const double invN = 1.0 / N;
    for (int l = 0; l < d; ++l) {
        if (l == k) { z[l] = {0.0, 0.0}; continue; }
        int ix;
        if (l < k) {
            if (dir == 1 && a >= s.ncb) ix = rand_index(it.seed, 3 + ctr, (uint64_t)(a - s.ncb), (uint64_t)l, N);
            else ix = it.Iset[((size_t)k * R + a) * d + l];
        } else {
            if (dir == 0 && b >= s.ncb) ix = rand_index(it.seed, 4 + ctr, (uint64_t)(b - s.ncb), (uint64_t)l, N);
            else ix = it.Jset[((size_t)(k + 1) * R + b) * d + l];
        }
        const double L = it.L[l];
        z[l] = {-L + (ix + 0.5) * 2.0 * L * invN, it.alpha[l]};
    }
    cplx e0 = {0.0, 0.0}, tau = {0.0, 0.0}, H = {1.0, 0.0}, zrest = {0.0, 0.0};
    cplx j0 = {0.0, 0.0}, tauj = {0.0, 0.0};       // the jump exponent's counterparts
    const bool strip = it.kind[0] == 3;
    for (int l = 0; l < d; ++l) {
        if (l == k) continue;
        zrest = cadd(zrest, z[l]);
        const double *Cl = it.C + l * d;
        cplx q = {0.0, 0.0};
        for (int l2 = 0; l2 < d; ++l2) {
            if (l2 == k) continue;
            q = {q.x + Cl[l2] * z[l2].x, q.y + Cl[l2] * z[l2].y};
        }
        const cplx w = {-0.5 * q.x, -it.m[l] - 0.5 * q.y};
        e0 = cadd(e0, cmul(z[l], w));
        tau = {tau.x - it.C[k * d + l] * z[l].x, tau.y - it.C[k * d + l] * z[l].y};
        H = cmul(H, factor(it.kind[l], z[l]));
        if (jumps) {
            const double *CJl = it.CJ + l * d;
            cplx qj = {0.0, 0.0};
            for (int l2 = 0; l2 < d; ++l2) {
                if (l2 == k) continue;
                qj = {qj.x + CJl[l2] * z[l2].x, qj.y + CJl[l2] * z[l2].y};
            }
            j0 = cadd(j0, cmul(z[l], {-0.5 * qj.x, -it.mJ[l] - 0.5 * qj.y}));
            tauj = {tauj.x - it.CJ[k * d + l] * z[l].x, tauj.y - it.CJ[k * d + l] * z[l].y};
        }
    }
    cplx *out = mode == 0 ? it.F : it.cores + (size_t)k * R * N * R;
    const int nc = s.nc;
    for (int i = 0; i < N; ++i) {
        const cplx zk = {-Lk + (i + 0.5) * etak, ak};
        cplx ex = cadd(cadd(e0, cmul(zk, tau)), ctab[i]);
        if (jumps) {
            const cplx g = cexp_(cadd(cadd(j0, cmul(zk, tauj)), jtab[i]));
            ex = cadd(ex, {it.lamT * (g.x - 1.0), it.lamT * g.y});
        }
        cplx v = cmul(cexp_(ex), cmul(H, htab[i]));
        if (strip) v = cmul(v, strip_joint(d, cadd(zrest, zk)));
        const size_t row = (dir == 0) ? (size_t)g * N + i : (size_t)i * ng + g;
        gst(out + row * nc + c, v);
    }
}

// Integrand at explicit multi-indices (verification entry point).
__global__ void k_eval_points(const Item *items, long long npts, const int *idx, cplx *out)
{
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const Item &it = items[0];
    out[p] = integrand(it, idx + p * it.d);
}

// ------------------------------------------------------------------ Householder R in LDS
// Triangularises an nr x nc block in LDS (a leaf block row-major with an odd row stride ncp, so
// that both a row and a column spread over the LDS banks; a merge's stacked factors packed by
// rows; both reached through a row-layout object) by Householder reflections
// H = I - tau w w^H, in panels of TSQR_NB columns. A panel is factored inside one wave (wave 0), one panel ahead of
// the trailing update that the other waves carry out (see householder_lds). The panel width
// trades wave 0's chain (narrow panels: fewer column applications per column) against barriers
// and the trailing update (wide panels). With 16-wave workgroups two columns measured fastest
// (71.4 options/s on the d = 5 headline batch of 192 options, against 70.7, 70.3 and 67.4 for
// one, three and four); with 8 waves one column had been (47.7 against 46.4 at 64 options).
// tri > 0: the block stacks tri upper-triangular nc x nc factors (a merge of the reduction
// tree); the reflector of column j then touches only row j of the first factor and rows 0..j of
// the others, and only those rows are visited. On exit row j of R is (alph[j], entries j+1..nc-1
// of row j).

// Row addressing of the block being triangularised: row(r) of a stacked row index r (as from
// hh_row) is a pointer p with p[c] the entry (r, c).
struct RowsPadded {                               // row-major, odd row stride ncp
    cplx *A;
    int ncp;
    __device__ __forceinline__ cplx *row(int r) const { return A + (size_t)r * ncp; }
};
// Stacked upper-triangular nc x nc factors, each packed by rows (row i holds columns i..nc-1,
// tp = nc (nc + 1) / 2 entries a factor): a merge of the reduction tree touches only entries
// (i, c) with c >= i, and up to four factors of 68 columns fit where two unpacked ones did.
struct RowsPacked {
    cplx *A;
    int nc, tp;
    __device__ __forceinline__ cplx *row(int r) const
    {
        const int b = r / nc, i = r - b * nc;
        return A + (size_t)b * tp + i * nc - (i * (i - 1)) / 2 - i;
    }
};

constexpr int TSQR_NB = 2;

__device__ __forceinline__ int hh_len(int j, int nr, int nc, int tri) { return tri ? 1 + (tri - 1) * (j + 1) : nr - j; }
__device__ __forceinline__ int hh_row(int k, int j, int nc, int tri)
{
    if (!tri) return j + k;
    if (k == 0) return j;
    const int q = (k - 1) / (j + 1);
    return nc * (1 + q) + (k - 1 - q * (j + 1));
}

// Orders one wave's LDS accesses across its lanes: a wave's LDS instructions execute in
// order, so only the compiler has to be kept from moving loads and stores across this point.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Rows per lane that the single-wave Householder steps keep in registers between their two
// passes (blocks up to 192 rows, which covers the leaves and merges of wide fibers); further
// rows are read again from LDS.
constexpr int HH_SLOTS = 3;

// reflector of column j over its support rows (one wave); see make_reflector. One pass sums the
// squared moduli of the entries below the leading one; when that sum and |x_j|^2 lie within
// [1e-290, 1e290] no square has overflowed and those that underflowed are negligible, and the
// reflector is formed from the unscaled column. Otherwise the largest magnitude is found, and the
// column is scaled by a power of two as in make_reflector (a column below 1e-280 is left as it
// is, tau = 0).
template <class L>
__device__ void make_reflector_rows(const L &Lr, int j, int len, int nc, int tri, cplx *alpha_out, double *tau_out)
{
    const int lane = threadIdx.x & 63;
    double sq = 0.0;
    cplx xv[HH_SLOTS];
    int xi[HH_SLOTS];
#pragma unroll
    for (int m = 0; m < HH_SLOTS; ++m) {
        const int k = lane + 64 * m;
        xi[m] = k < len ? hh_row(k, j, nc, tri) : 0;
        xv[m] = k < len ? Lr.row(xi[m])[j] : cplx{0.0, 0.0};
        if (k > 0) sq += cabs2(xv[m]);
    }
    for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) sq += cabs2(Lr.row(hh_row(k, j, nc, tri))[j]);
    sq = wave_sum(sq);
    const cplx x0 = Lr.row(j)[j];
    const double all = sq + cabs2(x0);
    ReflScalars r;
    if (all >= 1e-290 && all <= 1e290) {
        r = reflector_scalars(x0, 1.0, 0, sq);
    } else {
        double mx = 0.0;
#pragma unroll
        for (int m = 0; m < HH_SLOTS; ++m) mx = fmax(mx, fmax(fabs(xv[m].x), fabs(xv[m].y)));
        for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) {
            const cplx v = Lr.row(hh_row(k, j, nc, tri))[j];
            mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
        }
        mx = wave_max(mx);
        if (!(mx >= 1e-280) || !(mx <= 1e300)) {
            if (lane == 0) {
                *alpha_out = x0;
                *tau_out = 0.0;
            }
            return;
        }
        int e;
        frexp(mx, &e);
        const double sc = ldexp(1.0, -e);
        sq = 0.0;
#pragma unroll
        for (int m = 0; m < HH_SLOTS; ++m)
            if (lane + 64 * m > 0) sq += cabs2(cplx{xv[m].x * sc, xv[m].y * sc});
        for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) {
            const cplx v = Lr.row(hh_row(k, j, nc, tri))[j];
            sq += cabs2(cplx{v.x * sc, v.y * sc});
        }
        sq = wave_sum(sq);
        r = reflector_scalars(x0, sc, e, sq);
    }
#pragma unroll
    for (int m = 0; m < HH_SLOTS; ++m) {
        const int k = lane + 64 * m;
        if (k > 0 && k < len) Lr.row(xi[m])[j] = cmul(xv[m], r.cf);
    }
    for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) {
        cplx *p = Lr.row(hh_row(k, j, nc, tri)) + j;
        *p = cmul(*p, r.cf);
    }
    if (lane == 0) {
        Lr.row(j)[j] = {1.0, 0.0};
        *alpha_out = r.alpha;
        *tau_out = r.tau;
    }
}

// Applies reflectors j0..j1-1, in order, to columns [ca, cb). Threads t = 0..T-1 (T a multiple
// of 64, every one of them calling) form groups of S adjacent lanes, one pair of adjacent columns
// per group (w is read once for both), which split the columns' support rows; a dot product then
// needs an S-lane butterfly only.
template <class L>
__device__ void hh_apply_cols(const L &Lr, int nr, int nc, int tri, const double *tau,
                              int ca, int cb, int j0, int j1, int t, int T)
{
    const int nt = cb - ca;
    if (nt <= 0 || j1 <= j0) return;
    const int np = (nt + 1) / 2;                    // column pairs
    int S = 1;
    while (S < 16 && 2 * S * np <= T) S *= 2;
    const int sidx = t % S, per = T / S;
    for (int cq = 0; cq < np; cq += per) {
        const int cp = cq + t / S;
        const bool act = cp < np, hasB = act && 2 * cp + 1 < nt;
        const int cA = ca + (act ? 2 * cp : 0), cB = hasB ? cA + 1 : cA;
        for (int j = j0; j < j1; ++j) {
            const double tj = tau[j];
            if (tj == 0.0) continue;                // same for every lane
            const int len = hh_len(j, nr, nc, tri);
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            if (act)
                for (int k = sidx; k < len; k += S) {
                    const cplx *row = Lr.row(hh_row(k, j, nc, tri));
                    const cplx w = row[j];
                    const cplx p = cmulc(w, row[cA]), q = cmulc(w, row[cB]);
                    ar += p.x;
                    ai += p.y;
                    br += q.x;
                    bi += q.y;
                }
            ar = seg_sum(ar, S);
            ai = seg_sum(ai, S);
            br = seg_sum(br, S);
            bi = seg_sum(bi, S);
            const cplx fA = {tj * ar, tj * ai}, fB = {tj * br, tj * bi};
            if (act)
                for (int k = sidx; k < len; k += S) {
                    cplx *row = Lr.row(hh_row(k, j, nc, tri));
                    const cplx w = row[j];
                    const cplx x = row[cA], y = row[cB];
                    row[cA] = csub(x, cmul(fA, w));
                    if (hasB) row[cB] = csub(y, cmul(fB, w));
                }
        }
    }
}

// Applies reflectors j0..j1-1, in order, to the NQ <= TSQR_NB columns ca..ca+NQ-1, within the
// calling wave: each lane takes every 64th support row for all NQ columns, so one pass over the
// rows forms the NQ dot products (reduced across the wave together) and a second one updates;
// the first HH_SLOTS rows of a lane stay in registers between the passes.
template <int NQ, class L>
__device__ void hh_apply_wave_n(const L &Lr, int nr, int nc, int tri, const double *tau, int ca, int j0, int j1)
{
    constexpr int NV = NQ == 3 ? 8 : 2 * NQ;     // sums per reflector (real and imaginary parts)
    const int lane = threadIdx.x & 63;
    for (int j = j0; j < j1; ++j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;                    // same for every lane
        const int len = hh_len(j, nr, nc, tri);
        double sums[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) sums[q] = 0.0;
        cplx wv[HH_SLOTS], cv[HH_SLOTS][NQ];
        int ri[HH_SLOTS];
#pragma unroll
        for (int m = 0; m < HH_SLOTS; ++m) {
            const int k = lane + 64 * m;
            const bool in = k < len;
            ri[m] = in ? hh_row(k, j, nc, tri) : 0;
            const cplx *row = Lr.row(ri[m]);
            wv[m] = in ? row[j] : cplx{0.0, 0.0};
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                cv[m][q] = in ? row[ca + q] : cplx{0.0, 0.0};
                const cplx p = cmulc(wv[m], cv[m][q]);
                sums[q] += p.x;
                sums[NV / 2 + q] += p.y;
            }
        }
        for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) {
            const cplx *row = Lr.row(hh_row(k, j, nc, tri));
            const cplx w = row[j];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const cplx p = cmulc(w, row[ca + q]);
                sums[q] += p.x;
                sums[NV / 2 + q] += p.y;
            }
        }
        wave_sum_n<NV>(sums);
        cplx f[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = {tj * sums[q], tj * sums[NV / 2 + q]};
#pragma unroll
        for (int m = 0; m < HH_SLOTS; ++m)
            if (lane + 64 * m < len) {
                cplx *row = Lr.row(ri[m]);
#pragma unroll
                for (int q = 0; q < NQ; ++q) row[ca + q] = csub(cv[m][q], cmul(f[q], wv[m]));
            }
        for (int k = lane + 64 * HH_SLOTS; k < len; k += 64) {
            cplx *row = Lr.row(hh_row(k, j, nc, tri));
            const cplx w = row[j];
#pragma unroll
            for (int q = 0; q < NQ; ++q) row[ca + q] = csub(row[ca + q], cmul(f[q], w));
        }
        wave_lds_order();                           // reflector j+1 visits other rows per lane
    }
}
template <class L>
__device__ __forceinline__ void hh_apply_wave(const L &Lr, int nr, int nc, int tri, const double *tau,
                                              int ca, int n, int j0, int j1)
{
    static_assert(TSQR_NB >= 1 && TSQR_NB <= 4, "column counts 1..4");
    // only the widths a panel of TSQR_NB columns can ask for are instantiated (registers)
    if constexpr (TSQR_NB >= 4) if (n == 4) hh_apply_wave_n<4>(Lr, nr, nc, tri, tau, ca, j0, j1);
    if constexpr (TSQR_NB >= 3) if (n == 3) hh_apply_wave_n<3>(Lr, nr, nc, tri, tau, ca, j0, j1);
    if constexpr (TSQR_NB >= 2) if (n == 2) hh_apply_wave_n<2>(Lr, nr, nc, tri, tau, ca, j0, j1);
    if (n == 1) hh_apply_wave_n<1>(Lr, nr, nc, tri, tau, ca, j0, j1);
}

// Factors the panel of columns c..c+n-1 (n <= TSQR_NB) within the calling wave: each
// reflector is formed and then applied to the panel's later columns.
template <class L>
__device__ void hh_factor_panel_wave(const L &Lr, int nr, int nc, int tri, cplx *alph, double *tau, int c, int n)
{
    for (int j = c; j < c + n; ++j) {
        make_reflector_rows(Lr, j, hh_len(j, nr, nc, tri), nc, tri, &alph[j], &tau[j]);
        wave_lds_order();
        hh_apply_wave(Lr, nr, nc, tri, tau, j + 1, c + n - j - 1, j, j + 1);
    }
}

// Triangularises A in panels of TSQR_NB columns with a one-panel look-ahead: while the other
// waves apply panel P's reflectors to the columns beyond panel P+1, wave 0 applies them to
// panel P+1's columns and factors panel P+1 by itself. The two parts touch disjoint columns
// and read panel P's reflectors only, so one barrier per panel separates the steps.
template <class L>
__device__ void householder_lds(const L &Lr, int nr, int nc, int tri, cplx *alph, double *tau)
{
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int jmax = nr < nc ? nr : nc;
    const int t0 = nw > 1 ? 64 : 0;                 // first thread of the trailing update
    if (jmax > 0 && wave == 0) hh_factor_panel_wave(Lr, nr, nc, tri, alph, tau, 0, min(TSQR_NB, jmax));
    __syncthreads();
    for (int j0 = 0; j0 < jmax; j0 += TSQR_NB) {
        const int j1 = min(j0 + TSQR_NB, jmax);     // panel P: reflectors j0..j1-1 are formed
        const int n1 = min(TSQR_NB, jmax - j1);     // width of panel P+1 (0 at the end)
        if (wave == 0 && n1 > 0) {
            hh_apply_wave(Lr, nr, nc, tri, tau, j1, n1, j0, j1);
            hh_factor_panel_wave(Lr, nr, nc, tri, alph, tau, j1, n1);
        }
        if ((int)threadIdx.x >= t0)
            hh_apply_cols(Lr, nr, nc, tri, tau, j1 + n1, nc, j0, j1, threadIdx.x - t0, blockDim.x - t0);
        __syncthreads();
    }
}

// number of TSQR blocks at a level
__device__ __forceinline__ int tsqr_count(int rows, int BR, int G, int level)
{
    int n = (rows + BR - 1) / BR;
    for (int l = 0; l < level; ++l) n = (n + G - 1) / G;
    return n;
}
__device__ __forceinline__ int tsqr_final_level(int rows, int BR, int G)
{
    int n = (rows + BR - 1) / BR, l = 0;
    while (n > 1) { n = (n + G - 1) / G; ++l; }
    return l;
}

// One TSQR level: level 0 reduces row blocks of the fiber (BR rows, padded row-major in LDS),
// level L > 0 groups of G triangular factors of level L-1 (packed by rows in LDS). Writes
// nc x nc factors into buffer (level % 2).
__global__ __launch_bounds__(TSQR_THREADS) void k_tsqr(Item *items, ItemList work, int t, int dir, int level, int BR, int G)
{
    extern __shared__ cplx lds[];
    __shared__ cplx alph[MAXNC];
    __shared__ double tau[MAXNC];
    const int item = work.item(blockIdx.y);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int nc = s.nc;
    if (level > 0 && tsqr_count(s.rows, BR, G, level - 1) == 1) return;
    const int ncur = tsqr_count(s.rows, BR, G, level);
    const int blk = blockIdx.x;
    if (blk >= ncur) return;
    if (level == 0 && blk == 0 && threadIdx.x == 0) {
        const double m = s.rows, n = nc;
        it.work[TTFP_KERNEL_TSQR] += 8.0 * m * n * n - 8.0 / 3.0 * n * n * n;
    }
    const size_t rsz = (size_t)nc * nc;
    const int ncp = nc | 1;                          // odd row stride of a leaf block in LDS
    const int tp = nc * (nc + 1) / 2;                // entries of a packed triangular factor
    cplx *A = lds;
    int nr, tri = 0;
    const cplx *src;
    if (level == 0) {
        const int r0 = blk * BR;
        nr = min(BR, s.rows - r0);
        src = it.F + (size_t)r0 * nc;
    } else {
        const int nprev = tsqr_count(s.rows, BR, G, level - 1);
        const int g0 = blk * G, g1 = min(nprev, g0 + G);
        nr = (g1 - g0) * nc;
        tri = g1 - g0;                               // stacked triangular factors
        src = it.Rlev + (size_t)((level - 1) & 1) * it.nblk_max * rsz + (size_t)g0 * rsz;
    }
    if (level == 0) {
        // coalesced read of nr row-major rows into the padded row-major LDS block
        for (int e = threadIdx.x; e < nr * nc; e += blockDim.x) {
            const int i = e / nc, c = e % nc;
            A[(size_t)i * ncp + c] = src[e];
        }
    } else {
        // the upper triangles of the tri factors, packed by rows
        for (int e = threadIdx.x; e < tri * (int)rsz; e += blockDim.x) {
            const int b = e / (int)rsz, w = e - b * (int)rsz, i = w / nc, c = w - i * nc;
            if (c >= i) A[(size_t)b * tp + i * nc - (i * (i - 1)) / 2 + (c - i)] = src[e];
        }
    }
    __syncthreads();
    if (level == 0)
        householder_lds(RowsPadded{A, ncp}, nr, nc, 0, alph, tau);
    else
        householder_lds(RowsPacked{A, nc, tp}, nr, nc, tri, alph, tau);
    cplx *dst = it.Rlev + (size_t)(level & 1) * it.nblk_max * rsz + (size_t)blk * rsz;
    const int jmax = nr < nc ? nr : nc;
    for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
        int j = e / nc, c = e % nc;
        cplx v = {0.0, 0.0};
        if (j < jmax && c >= j) {
            // row j of R: the first factor's row j
            const cplx *rowj = level == 0 ? A + (size_t)j * ncp : A + j * nc - (j * (j - 1)) / 2 - j;
            v = (c == j) ? alph[j] : rowj[c];
        }
        dst[e] = v;
    }
}

// ------------------------------------------------------------------ Cholesky QR on the matrix cores
// The triangular factor of the fiber F (m x nc) by three passes of shifted Cholesky QR (Fukaya,
// Kannan, Nakatsukasa, Yamamoto and Yanagisawa, "Shifted Cholesky QR for computing the QR
// factorization of ill-conditioned matrices", 2020):
//   pass 0: G = (sF)^H (sF) with s = 2^-e (e from the largest entry), R0 = chol(G + shift I)
//   pass 1: Q = sF R0^{-1},  R1 = chol(Q^H Q + shift I)
//   pass 2: Q <- Q R1^{-1},  R2 = chol(Q^H Q + shift I);   R = R2 R1 R0 / s
// (or two passes, R = R1 R0 / s, a tuning choice).
// A pass resolves the singular values that stand above the square root of its shift; the next
// pass sees them relative to what is left, so three passes resolve the spectrum well below the
// rank threshold while R^H R = F^H F holds to about the shift (10 nc u relative, with the Gram
// accumulated in FP64). Rank-deficient fibers (exact zero columns, saturated ranks) are covered
// by the shift of every pass; a Cholesky that still meets a non-positive pivot is redone with a
// hundred times the shift. The Gram products and the triangular transforms are dense
// contractions over the fiber's rows and run on the FP64 matrix cores (v_mfma_f64_16x16x4f64);
// the nc x nc Cholesky, inverse and factor product are one small workgroup per item.
constexpr int GRAM_ROWS = 1024;                    // fiber rows per Gram workgroup
constexpr int GRAM_CHUNK = 32;                     // rows staged in LDS at a time
constexpr int NCPAD = (MAXNC + 15) / 16 * 16;      // columns rounded up to whole 16-wide tiles
constexpr int GRAM_NOSCALE = -100000;              // block exponent of a block of zeros
typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int gram_blocks(int rows) { return (rows + GRAM_ROWS - 1) / GRAM_ROWS; }

// Partial Gram of one block of GRAM_ROWS fiber rows: P = X^H X over the block's rows, upper
// 16 x 16 tiles only, written to it.Gp[block] (nc x nc, row-major). Pass 0 reads F and scales
// it by 2^-e_blk, e_blk the exponent of the largest entry seen so far in the block (the
// accumulators are rescaled exactly when a later chunk raises it; e_blk goes to it.Ge[block]);
// passes 1 and 2 read Q unscaled. A chunk of rows is staged in LDS as separate real and
// imaginary planes whose row stride (NCPAD doubles, 32 banks mod 64) lets the two rows a half
// wave reads fall on disjoint banks; the next chunk is loaded into registers meanwhile. Each wave
// takes one or two tiles (GRAM_THREADS below). Complex products by three real ones (Gauss): with X = Xr + i Xi,
// Y = Yr + i Yi, X^H Y = (t1 + t2) + i (t3 - t1 + t2), t1 = Xr^T Yr, t2 = Xi^T Yi,
// t3 = (Xr - Xi)^T (Yr + Yi): three independent accumulators per tile.
// GRAM_THREADS 512 (two tiles per wave) or 1024 (one tile per wave: half the critical path of a
// chunk): a launch tuning that leaves every result bit unchanged (each tile sums the same rows in
// the same order).
template <int GRAM_THREADS>
__global__ __launch_bounds__(GRAM_THREADS, GRAM_THREADS == 1024 ? 8 : 4) void k_gram(Item *items, ItemList work, int t, int dir, int pass)
{
    constexpr int PER = (GRAM_CHUNK * MAXNC + GRAM_THREADS - 1) / GRAM_THREADS;   // chunk entries per thread
    constexpr int NW = GRAM_THREADS / 64, TPW = 1024 / GRAM_THREADS;               // waves, tiles per wave
    __shared__ double cre[GRAM_CHUNK][NCPAD], cim[GRAM_CHUNK][NCPAD];
    __shared__ double wmax[NW];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int m = s.rows, nc = s.nc, blk = blockIdx.y;
    if (blk >= gram_blocks(m)) return;
    if (blk == 0 && threadIdx.x == 0) it.work[TTFP_KERNEL_GRAM] += 4.0 * m * (double)nc * nc;
    const cplx *src = pass == 0 ? it.F : it.Qb;
    const int T = (nc + 15) / 16, ntiles = T * (T + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // this wave's tiles: q = wave, wave + NW in the order (0,0) (0,1) .. (0,T-1) (1,1) ..
    int tI[TPW], tJ[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        int q = wave + NW * u, I = 0;
        while (I < T && q >= T - I) { q -= T - I; ++I; }
        tI[u] = I;
        tJ[u] = I + q;
    }
    const int nt = ntiles > wave ? min(TPW, (ntiles - wave + NW - 1) / NW) : 0;
    // entry e = tid + GRAM_THREADS q of a chunk is row e / nc, column e % nc (rows of a chunk are
    // contiguous in the fiber, so a chunk is one coalesced sweep); lo[q] is its place in the LDS
    // planes, -1 past the chunk
    int lo[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + GRAM_THREADS * q, er = e / nc;
        lo[q] = er < GRAM_CHUNK ? er * NCPAD + (e - er * nc) : -1;
    }
    // padding columns nc .. 16 T - 1 stay zero for every chunk
    for (int e = tid; e < GRAM_CHUNK * 16 * T; e += GRAM_THREADS) {
        const int c = e % (16 * T);
        if (c >= nc) {
            cre[e / (16 * T)][c] = 0.0;
            cim[e / (16 * T)][c] = 0.0;
        }
    }
    double4_t p1[TPW], p2[TPW], p3[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        p1[u] = double4_t{0.0, 0.0, 0.0, 0.0};
        p2[u] = p1[u];
        p3[u] = p1[u];
    }
    int e_blk = GRAM_NOSCALE;
    double sc = 1.0;
    const int r0 = blk * GRAM_ROWS, r1 = min(m, r0 + GRAM_ROWS);
    cplx pre[PER];
    auto fetch = [&](int c0) {
        const int n = min(GRAM_CHUNK, r1 - c0) * nc;
        const cplx *g = src + (size_t)c0 * nc;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + GRAM_THREADS * q;
            pre[q] = e < n ? gld(g + e) : cplx{0.0, 0.0};
        }
    };
    fetch(r0);
    for (int c0 = r0; c0 < r1; c0 += GRAM_CHUNK) {
        const int nr = min(GRAM_CHUNK, r1 - c0);
        if (pass == 0) {
            double mx = 0.0;
#pragma unroll
            for (int q = 0; q < PER; ++q) mx = fmax(mx, fmax(fabs(pre[q].x), fabs(pre[q].y)));
            mx = wave_max(mx);
            if (lane == 0) wmax[wave] = mx;
        }
        __syncthreads();                         // the previous chunk has been multiplied
        if (pass == 0) {
            double mx = wave_max(lane < NW ? wmax[lane] : 0.0);
            if (mx > 0.0) {
                int e;
                frexp(mx, &e);
                if (e > e_blk) {
                    if (e_blk != GRAM_NOSCALE) {
                        const double f = ldexp(1.0, 2 * (e_blk - e));
#pragma unroll
                        for (int u = 0; u < TPW; ++u) {
                            p1[u] *= f;
                            p2[u] *= f;
                            p3[u] *= f;
                        }
                    }
                    e_blk = e;
                    sc = ldexp(1.0, -e);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (lo[q] >= 0) {                        // rows past nr were loaded as zeros
                (&cre[0][0])[lo[q]] = pre[q].x * sc;
                (&cim[0][0])[lo[q]] = pre[q].y * sc;
            }
        __syncthreads();
        if (c0 + GRAM_CHUNK < r1) fetch(c0 + GRAM_CHUNK);
        const int nks = (nr + 3) / 4;
        for (int ks = 0; ks < nks; ++ks) {
            const int row = 4 * ks + lk;
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                if (u >= nt) break;
                const double xr = cre[row][16 * tI[u] + li], xi = cim[row][16 * tI[u] + li];
                const double yr = cre[row][16 * tJ[u] + li], yi = cim[row][16 * tJ[u] + li];
                p1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, yr, p1[u], 0, 0, 0);
                p2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, yi, p2[u], 0, 0, 0);
                p3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr - xi, yr + yi, p3[u], 0, 0, 0);
            }
        }
    }
    cplx *P = it.Gp + (size_t)blk * nc * nc;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        if (u >= nt) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * tI[u] + lk + 4 * v, j = 16 * tJ[u] + li;
            if (i < nc && j < nc && i <= j) P[(size_t)i * nc + j] = {p1[u][v] + p2[u][v], p3[u][v] - p1[u][v] + p2[u][v]};
        }
    }
    if (tid == 0) it.Ge[blk] = pass == 0 ? e_blk : 0;
}
template __global__ void k_gram<512>(Item *, ItemList, int, int, int);
template __global__ void k_gram<1024>(Item *, ItemList, int, int, int);

// Packed upper-triangular storage of an n x n matrix: row i starts at i n - i (i - 1) / 2.
__device__ __forceinline__ int up_off(int i, int n) { return i * n - (i * (i - 1)) / 2; }
// row of packed entry e: the largest i with up_off(i) <= e (from the quadratic, then corrected)
__device__ __forceinline__ int up_row(int e, int n)
{
    const double b = 2.0 * n + 1.0;
    int i = (int)(0.5 * (b - sqrt(b * b - 8.0 * e)));
    i = max(0, min(i, n - 1));
    while (i > 0 && up_off(i, n) > e) --i;
    while (i + 1 < n && up_off(i + 1, n) <= e) ++i;
    return i;
}

// Sums the partial Grams (scaled to the largest block exponent), factors G + shift I = R^H R
// (upper, real positive diagonal), forms X = R^{-1} for the next transform (it.Xf, nc x nc
// row-major with zeros below the diagonal) and the running factor it.Rf: R in pass 0, R Rf after.
// The last pass leaves Rf / s = the triangular factor of F (nc x nc, row-major), which the
// column-pivoted QR reads.
__global__ __launch_bounds__(256) void k_chol(Item *items, ItemList work, int t, int dir, int pass, int last)
{
    __shared__ cplx Rp[MAXNC * (MAXNC + 1) / 2];   // G, then its Cholesky factor (packed upper)
    __shared__ cplx Xp[MAXNC * (MAXNC + 1) / 2];   // R^{-1}, then the factor product (packed upper)
    __shared__ double red[256 / 64];
    __shared__ int sh_fail;
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int m = s.rows, nc = s.nc, nb = gram_blocks(m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nthr = blockDim.x;
    const int np = nc * (nc + 1) / 2;
    // common exponent of the partials (pass 0), then their sum in block order
    int emax = GRAM_NOSCALE;
    if (pass == 0)
        for (int b = 0; b < nb; ++b) emax = max(emax, it.Ge[b]);
    else
        emax = 0;
    double tr = 0.0;
    for (int e = threadIdx.x; e < np; e += nthr) {
        const int i = up_row(e, nc), j = i + (e - up_off(i, nc));
        cplx acc = {0.0, 0.0};
        if (emax != GRAM_NOSCALE)
            for (int b = 0; b < nb; ++b) {
                const int eb = it.Ge[b];
                if (eb == GRAM_NOSCALE) continue;
                const double f = ldexp(1.0, 2 * (eb - emax));
                const cplx g = it.Gp[(size_t)b * nc * nc + (size_t)i * nc + j];
                acc = {acc.x + f * g.x, acc.y + f * g.y};
            }
        Xp[e] = acc;                               // G kept here for retries
        if (i == j) tr += acc.x;
    }
    tr = wave_sum(tr);
    if (lane == 0) red[wave] = tr;
    __syncthreads();
    tr = 0.0;
    for (int w = 0; w < nthr / 64; ++w) tr += red[w];
    double shift = 10.0 * nc * 2.220446049250313e-16 * tr;
    // Cholesky of G + shift I (right-looking, packed rows; the trailing rows of a step spread over
    // the waves, their columns over the lanes), redone with a larger shift after a non-positive
    // pivot
    const int nw = nthr / 64;
    for (int attempt = 0; attempt < 6; ++attempt) {
        for (int e = threadIdx.x; e < np; e += nthr) Rp[e] = Xp[e];
        __syncthreads();
        for (int i = threadIdx.x; i < nc; i += nthr) Rp[up_off(i, nc)].x += shift;
        __syncthreads();
        int fail = 0;
        for (int j = 0; j < nc; ++j) {
            const int oj = up_off(j, nc);
            const double dj = Rp[oj].x;                 // the same value in every thread
            if (!(dj > 0.0) || !(dj < INFINITY)) { fail = 1; break; }
            const double rjj = sqrt(dj), inv = 1.0 / rjj;
            for (int k = j + 1 + threadIdx.x; k < nc; k += nthr) Rp[oj + k - j] = {Rp[oj + k - j].x * inv, Rp[oj + k - j].y * inv};
            __syncthreads();
            if (threadIdx.x == 0) Rp[oj] = {rjj, 0.0};
            // trailing update of rows i > j: R_ik -= conj(R_ji) R_jk, k >= i
            for (int ii = j + 1 + wave; ii < nc; ii += nw) {
                const cplx rji = Rp[oj + ii - j];
                const int oi = up_off(ii, nc);
                for (int kk = ii + lane; kk < nc; kk += 64) {
                    cplx &w = Rp[oi + kk - ii];
                    w = csub(w, cmulc(rji, Rp[oj + kk - j]));
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) sh_fail = fail;
        __syncthreads();
        if (!sh_fail) break;
        if (tr <= 0.0 || !(tr < INFINITY)) break;
        shift = shift > 0.0 ? 100.0 * shift : 1e-300;
        __syncthreads();
    }
    if (sh_fail || !(tr > 0.0)) {
        // a zero (or non-finite) fiber: factor zero, transform zero
        for (int e = threadIdx.x; e < np; e += nthr) Rp[e] = {0.0, 0.0};
        __syncthreads();
    }
    // X = R^{-1} (only the transform of the next pass needs it), a row at a time from the bottom:
    // row l of R X = I gives X_lc = (delta_lc - sum_{k>l} R_lk X_kc) / R_ll, and once row l is
    // known its terms leave the rows above it (rows over the waves, columns over the lanes). A
    // zero diagonal entry R_cc (a zero fiber column) gives a zero column of X.
    if (!last) {
        for (int e = threadIdx.x; e < np; e += nthr) Xp[e] = {0.0, 0.0};
        __syncthreads();
        for (int l = nc - 1; l >= 0; --l) {
            const int ol = up_off(l, nc);
            const double rll = Rp[ol].x;
            for (int c = l + threadIdx.x; c < nc; c += nthr) {
                const cplx tlc = Xp[ol + c - l];
                const double v = c == l ? 1.0 : 0.0;
                const bool zero = rll == 0.0 || Rp[up_off(c, nc)].x == 0.0;
                Xp[ol + c - l] = zero ? cplx{0.0, 0.0} : cplx{(v + tlc.x) / rll, tlc.y / rll};
            }
            __syncthreads();
            for (int i = wave; i < l; i += nw) {
                const int oi = up_off(i, nc);
                const cplx ril = Rp[oi + l - i];
                for (int c = l + lane; c < nc; c += 64) {
                    cplx &x = Xp[oi + c - i];
                    x = csub(x, cmul(ril, Xp[ol + c - l]));
                }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < nc * nc; e += nthr) {
            const int i = e / nc, j = e % nc;
            it.Xf[e] = j >= i ? Xp[up_off(i, nc) + j - i] : cplx{0.0, 0.0};
        }
    }
    // running factor: Rf <- R (pass 0) or R Rf (the previous Rf staged in Xp, packed); the last
    // pass also undoes the scaling
    const double unscale = last ? ldexp(1.0, it.gram_e == GRAM_NOSCALE ? 0 : it.gram_e) : 1.0;
    constexpr int PER = (MAXNC * (MAXNC + 1) / 2 + 255) / 256;
    cplx res[PER];
    if (pass > 0) {
        __syncthreads();                           // Xf written from Xp
        for (int e = threadIdx.x; e < np; e += nthr) {
            const int i = up_row(e, nc), j = i + (e - up_off(i, nc));
            Xp[e] = it.Rf[(size_t)i * nc + j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e >= np) break;
        const int i = up_row(e, nc), j = i + (e - up_off(i, nc)), oi = up_off(i, nc);
        cplx acc;
        if (pass == 0) {
            acc = Rp[e];
        } else {
            acc = {0.0, 0.0};
            for (int l = i; l <= j; ++l) acc = cadd(acc, cmul(Rp[oi + l - i], Xp[up_off(l, nc) + j - l]));
        }
        res[q] = {acc.x * unscale, acc.y * unscale};
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e >= np) break;
        const int i = up_row(e, nc), j = i + (e - up_off(i, nc));
        it.Rf[(size_t)i * nc + j] = res[q];
    }
    for (int e = threadIdx.x; e < nc * nc; e += nthr) {
        const int i = e / nc, j = e % nc;
        if (j < i) it.Rf[e] = {0.0, 0.0};
    }
    if (pass == 0 && threadIdx.x == 0) it.gram_e = emax;
}

// Q = X_src Xf for every fiber row, in 16-row panels per wave on the FP64 matrix cores: pass 1
// reads F scaled by 2^-gram_e and writes Q; pass 2 transforms Q in place (a wave owns its panel,
// and every load of the panel precedes the panel's stores). Xf is upper triangular, so output
// column tile J takes only k < 16 (J + 1). Xf sits in LDS as real and imaginary planes with a row
// stride of NCPAD doubles (the two k-rows a half wave reads fall on disjoint banks); complex
// products by three real ones (Gauss) into three independent accumulators per tile.
constexpr int XF_WAVES = 12;                       // 16-row panels per workgroup
__global__ __launch_bounds__(64 * XF_WAVES) void k_xform(Item *items, ItemList work, int t, int dir, int pass)
{
    __shared__ double Xr[MAXNC][NCPAD], Xi[MAXNC][NCPAD];
    const int item = work.item(blockIdx.y);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int nc = s.nc, m = s.rows;
    if (blockIdx.x * 16 * XF_WAVES >= m) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) it.work[TTFP_KERNEL_XFORM] += 4.0 * m * (double)nc * nc;
    const int T = (nc + 15) / 16;
    for (int e = threadIdx.x; e < nc * 16 * T; e += blockDim.x) {
        const int k = e / (16 * T), c = e - k * 16 * T;
        const cplx x = c < nc ? it.Xf[(size_t)k * nc + c] : cplx{0.0, 0.0};
        Xr[k][c] = x.x;
        Xi[k][c] = x.y;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int row0 = blockIdx.x * 16 * XF_WAVES + wave * 16;
    if (row0 >= m) return;
    const cplx *src = pass == 1 ? it.F : it.Qb;
    const double sc = pass == 1 ? ldexp(1.0, it.gram_e == GRAM_NOSCALE ? 0 : -it.gram_e) : 1.0;
    double4_t prr[NCPAD / 16], pii[NCPAD / 16], pss[NCPAD / 16];
#pragma unroll
    for (int q = 0; q < NCPAD / 16; ++q) {
        prr[q] = double4_t{0.0, 0.0, 0.0, 0.0};
        pii[q] = prr[q];
        pss[q] = prr[q];
    }
    const int arow = row0 + li;
    // the left operand of the next k-step is loaded while this one's products run
    cplx an = (arow < m && lk < nc) ? gld(src + (size_t)arow * nc + lk) : cplx{0.0, 0.0};
    for (int k0 = 0; k0 < nc; k0 += 4) {
        const int kk = k0 + lk;
        const cplx a = an;
        if (k0 + 4 < nc) an = (arow < m && kk + 4 < nc) ? gld(src + (size_t)arow * nc + kk + 4) : cplx{0.0, 0.0};
        const double ar = a.x * sc, ai = a.y * sc, as = ar + ai;
        const int kr = kk < nc ? kk : 0;           // rows of Xf past nc: the operand is zero anyway
#pragma unroll
        for (int q = 0; q < NCPAD / 16; ++q) {
            if (q >= T) break;
            if (k0 >= 16 * (q + 1)) continue;     // rows of X below the diagonal block are zero
            const double br = Xr[kr][16 * q + li], bi = Xi[kr][16 * q + li];
            prr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, prr[q], 0, 0, 0);
            pii[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, pii[q], 0, 0, 0);
            pss[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, br + bi, pss[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = row0 + lk + 4 * v;
#pragma unroll
        for (int q = 0; q < NCPAD / 16; ++q) {
            if (q >= T) break;
            const int col = 16 * q + li;
            if (row < m && col < nc)
                gst(it.Qb + (size_t)row * nc + col, cplx{prr[q][v] - pii[q][v], pss[q][v] - prr[q][v] - pii[q][v]});
        }
    }
}

// ------------------------------------------------------------------ pivoted QR of R, rank, inverse
__global__ __launch_bounds__(QRCP_THREADS) void k_qrcp(Item *items, ItemList work, int t, int dir, int BR, int G)
{
    __shared__ cplx A[MAXNC * (MAXNC | 1)];
    __shared__ double nrm[MAXNC];
    __shared__ double tauq[MAXNC];
    __shared__ int perm[MAXNC];
    __shared__ cplx alph[MAXNC];
    __shared__ int shi[4];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int nc = s.nc, ncp = nc | 1;              // odd row stride in LDS
    const int nthr = blockDim.x;
    const size_t rsz = (size_t)nc * nc;
    // the fiber's triangular factor: from the Cholesky QR (BR == 0) or the last TSQR level
    const cplx *src = BR == 0 ? it.Rf : it.Rlev + (size_t)(tsqr_final_level(s.rows, BR, G) & 1) * it.nblk_max * rsz;
    for (int e = threadIdx.x; e < nc * nc; e += nthr) A[(e / nc) * ncp + e % nc] = src[e];
    for (int c = threadIdx.x; c < nc; c += nthr) perm[c] = c;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < nc; ++j) {
        // trailing column norms over rows j..nc-1, groups of S lanes per column; formed from the
        // column scaled by its largest entry so that tiny columns keep their order instead of
        // underflowing to zero (outside [1e-280, 1e300] the largest entry itself orders it)
        {
            const int ncol = nc - j;
            int S = 1;
            while (S < 16 && 2 * S * ncol <= nthr) S *= 2;
            const int per = nthr / S, sidx = threadIdx.x % S;
            for (int cq = 0; cq < ncol; cq += per) {
                const int cl = cq + threadIdx.x / S;
                const bool act = cl < ncol;
                const int c = j + (act ? cl : 0);
                double mx = 0.0;
                if (act)
                    for (int i = j + sidx; i < nc; i += S)
                        mx = fmax(mx, fmax(fabs(A[i * ncp + c].x), fabs(A[i * ncp + c].y)));
                mx = seg_max(mx, S);
                const bool scaled = mx >= 1e-280 && mx <= 1e300;
                const double inv = scaled ? 1.0 / mx : 0.0;
                double q = 0.0;
                if (act)
                    for (int i = j + sidx; i < nc; i += S)
                        q += cabs2(cplx{A[i * ncp + c].x * inv, A[i * ncp + c].y * inv});
                q = seg_sum(q, S);
                if (act && sidx == 0) nrm[c] = scaled ? mx * sqrt(q) : mx;
            }
        }
        __syncthreads();
        // pivot (largest norm, lowest index on ties), column swap and reflector: wave 0
        if (wave == 0) {
            ArgMax bst = {-1.0, j};
            for (int c = j + lane; c < nc; c += 64) bst = better(bst, ArgMax{nrm[c], c});
            bst = wave_argmax(bst);
            const int p = bst.i;
            if (p != j) {
                for (int i = lane; i < nc; i += 64) {
                    const cplx tmp = A[i * ncp + j];
                    A[i * ncp + j] = A[i * ncp + p];
                    A[i * ncp + p] = tmp;
                }
                if (lane == 0) {
                    const int tp = perm[j];
                    perm[j] = perm[p];
                    perm[p] = tp;
                }
            }
            wave_lds_order();
            make_reflector(A + j, ncp, j, nc, &alph[j], &tauq[j]);
        }
        __syncthreads();
        hh_apply_cols(RowsPadded{A, ncp}, nc, nc, 0, tauq, j + 1, nc, j, j + 1, threadIdx.x, nthr);
        __syncthreads();
    }
    // rank: leading pivots above rank_eps * |R_00|
    if (threadIdx.x == 0) {
        const double r00 = hypot(alph[0].x, alph[0].y);
        int r = 0;
        while (r < nc && r00 > 0.0 && hypot(alph[r].x, alph[r].y) > it.rank_eps * r00) ++r;
        if (r < 1) r = 1;
        int cap = min(it.R, s.rows);
        if (dir == 2) cap = min(cap, nc);
        if (r > cap) {
            if (dir != 2) it.capped = 1;
            r = cap;
        }
        shi[1] = r;
    }
    __syncthreads();
    const int r = shi[1];
    // inverse of the leading r x r block of the pivoted factor (columns by back substitution).
    // The reflectors below the diagonal are no longer needed: entry (i, c), i <= c, of the inverse
    // is kept transposed at row c + 1, column i of A (c + 1 <= r <= MAXNC - 1 when r < nc, and
    // r <= 64 < nc otherwise), clear of the strict upper triangle that the substitution reads, so
    // that the kernel's LDS leaves room for two workgroups per CU.
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
        cplx *X = A + (c + 1) * ncp;               // column c of the inverse: X[i] = (R^-1)_{ic}
        cplx rcc = alph[c];
        X[c] = (rcc.x == 0.0 && rcc.y == 0.0) ? cplx{0.0, 0.0} : cdiv({1.0, 0.0}, rcc);
        for (int i = c - 1; i >= 0; --i) {
            cplx acc = {0.0, 0.0};
            for (int l = i + 1; l <= c; ++l) acc = cadd(acc, cmul(A[i * ncp + l], X[l]));
            cplx rii = alph[i];
            X[i] = (rii.x == 0.0 && rii.y == 0.0) ? cplx{0.0, 0.0} : cplx{-cdiv(acc, rii).x, -cdiv(acc, rii).y};
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int i = e / r, c = e - i * r;
        cplx v = {0.0, 0.0};
        if (i <= c) v = A[(c + 1) * ncp + i];
        it.Rinv[e] = v;
    }
    for (int c = threadIdx.x; c < r; c += blockDim.x) it.perm[c] = perm[c];
    if (threadIdx.x == 0) it.rsel = r;
}

// ------------------------------------------------------------------ basis of the kept columns
// Y = F[:, perm[:r]] R2^{-1} on the FP64 matrix cores, laid out as in k_interp (a wave forms a
// 16-row panel as up to four 16 x 16 complex tiles, three real MFMA products each); the
// triangular inverse is held in LDS with its zero lower part, and output tile q takes only the
// k-steps of rows k < 16 (q + 1). Each row's squared norm goes to
// its key (the start of maxvol reads them).
// PANEL_WAVES waves per workgroup (8 or 16) and PPW 16-row panels per wave (1 or 2): a launch
// tuning that leaves every result bit unchanged (a row's product does not depend on the workgroup
// or wave it falls in). More rows per workgroup spread the 64 KiB staging of R^-1 over more rows.
template <int PANEL_WAVES, int PPW>
__global__ __launch_bounds__(64 * PANEL_WAVES, 4) void k_basis(Item *items, ItemList work, int t, int dir)
{
    __shared__ cplx Ri[TTFP_MAX_RANK * TTFP_MAX_RANK];
    __shared__ int pm[TTFP_MAX_RANK];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int r = it.rsel, nc = s.nc, m = s.rows;
    const int rows_per_wg = 16 * PANEL_WAVES * PPW;
    if (blockIdx.y * rows_per_wg >= m) return;
    if (blockIdx.y == 0 && threadIdx.x == 0) it.work[TTFP_KERNEL_BASIS] += 4.0 * (double)m * r * r;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) Ri[e] = it.Rinv[e];
    for (int e = threadIdx.x; e < r; e += blockDim.x) pm[e] = it.perm[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
    for (int pp = 0; pp < PPW; ++pp) {
        const int row0 = blockIdx.y * rows_per_wg + (pp * PANEL_WAVES + wave) * 16;
        if (row0 >= m) break;
        const int li = lane & 15, lk = lane >> 4;
        const int ntile = (r + 15) / 16;
        // complex products by three real ones (Gauss): prr = Ar Br, pii = Ai Bi, pss = (Ar + Ai)(Br + Bi);
        // re = prr - pii, im = pss - prr - pii
        double4_t prr[4], pii[4], pss[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            prr[q] = double4_t{0.0, 0.0, 0.0, 0.0};
            pii[q] = double4_t{0.0, 0.0, 0.0, 0.0};
            pss[q] = double4_t{0.0, 0.0, 0.0, 0.0};
        }
        const int arow = row0 + li;
        // the left operand of the next k-step is loaded while this one's products run
        cplx an = (arow < m && lk < r) ? gld(it.F + (size_t)arow * nc + pm[lk]) : cplx{0.0, 0.0};
        // k-steps by 16-row blocks kb of R2^-1: block kb meets only the tiles q >= kb
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            if (kb >= ntile) break;
            for (int k0 = 16 * kb; k0 < min(r, 16 * kb + 16); k0 += 4) {
                const int kk = k0 + lk;
                const cplx a = an;
                if (k0 + 4 < r) an = (arow < m && kk + 4 < r) ? gld(it.F + (size_t)arow * nc + pm[kk + 4]) : cplx{0.0, 0.0};
#pragma unroll
                for (int q = kb; q < 4; ++q) {
                    if (q >= ntile) break;
                    const int jj = 16 * q + li;
                    const cplx b = (kk < r && jj < r) ? Ri[kk * r + jj] : cplx{0.0, 0.0};
                    prr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, prr[q], 0, 0, 0);
                    pii[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, pii[q], 0, 0, 0);
                    pss[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, pss[q], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + lk + 4 * v;
            double nrm = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= ntile) break;
                const int col = 16 * q + li;
                const cplx val = {prr[q][v] - pii[q][v], pss[q][v] - prr[q][v] - pii[q][v]};
                nrm += (row < m && col < r) ? cabs2(val) : 0.0;
                if (row < m && col < r) gst(it.Y + (size_t)row * r + col, val);
            }
            // the row's squared norm: the lane's columns li + 16 q, then the 16 lanes of the row
            nrm += __shfl_xor(nrm, 1, 64);
            nrm += __shfl_xor(nrm, 2, 64);
            nrm += __shfl_xor(nrm, 4, 64);
            nrm += __shfl_xor(nrm, 8, 64);
            if (row < m && li == 0) gst(it.keys + row, (float)nrm);
        }
    }
}
template __global__ void k_basis<8, 1>(Item *, ItemList, int, int);
template __global__ void k_basis<16, 1>(Item *, ItemList, int, int);
template __global__ void k_basis<8, 2>(Item *, ItemList, int, int);
template __global__ void k_basis<16, 2>(Item *, ItemList, int, int);

// ------------------------------------------------------------------ maxvol
// block-wide argmax (ties: lowest flat index); every thread receives the result: within each wave
// as above, across waves through LDS
__device__ ArgMax block_argmax(ArgMax a, ArgMax *scratch)
{
    a = wave_argmax(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();                     // earlier readers of scratch are done
    if (lane == 0) scratch[wave] = a;
    __syncthreads();
    ArgMax m = scratch[0];
    for (int w = 1; w < nw; ++w) m = better(m, scratch[w]);
    return m;
}

// Dominant r x r submatrix of Y (rows x r) and the interpolation matrix B = Y Y[piv]^{-1}.
//
// k_maxvol works on a block of candidate rows: the K = min(512, m) rows of largest norm (Y has
// orthonormal columns, so these are the rows of largest leverage).
//  1. start: from the second half sweep in a direction on, the pivots of the previous half sweep
//     in that direction mapped onto this fiber's rows, when all r of them map and their block is
//     not near-singular; otherwise Gaussian elimination with partial pivoting on the candidate
//     block (blocked by panels in LDS), continued over all m rows through their residuals when
//     the block is numerically rank deficient.
//  2. A^{-1} = Y[piv]^{-1} by Gauss-Jordan with partial pivoting (A in registers, A^{-1} in LDS),
//     and the block's rows of B, Bc = Y[cand] A^{-1}, on the matrix cores.
//  3. maxvol swaps on Bc: while its entry of largest modulus exceeds 1 + delta, that row
//     replaces the pivot of its column and Bc takes the rank-one update
//     Bc -= Bc[:,j] (Bc[i,:] - e_j) / Bc[i,j]. Each swap multiplies |det Y[piv]| by more than
//     1 + delta; at most 4 r + 16 swaps.
//  4. A^{-1} of the final pivots, stored for k_interp: the inverse of step 2 carried through
//     the swaps by the same rank-one updates (Sherman-Morrison), or recomputed by Gauss-Jordan
//     after more than MV_SM_MAX swaps; with it the largest squared column norm of A^{-1}.
// k_interp's checking passes form B for every row that the row bound does not clear (a tiled
// product spread over the whole chip) and mark the rows whose largest |B_ij| exceeds 1 + delta.
// k_maxvol_refine puts the pivots and the worst such rows into a new block and repeats 3-4,
// after which a checking pass runs again; when no row violates, both return at once. The result
// is dominant over every row once no row violates; k_interp's final pass stores B.
constexpr int MV_KMAX = 512;

// Up to K indices g < n of largest value v[g * stride] (nonnegative floats, largest vmax), among
// those of value >= lo0: the first ones in index order among those at or above a threshold
// found by bisection (stopped once between K and K + K / 8 values reach it), so that the choice
// does not depend on scheduling. Writes out[0..Kc) and returns Kc (same in every thread). Every
// thread of the workgroup must call it.
__device__ int select_largest(const float *v, int stride, int n, int K, float lo0, float vmax, int *out, ArgMax *red,
                              int *shi, float *shf)
{
    __shared__ int cntb[2][16];
    const int nthr = blockDim.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = nthr >> 6;
    __syncthreads();
    int par = 0;
    // number of values >= thr, in every thread (one barrier; the two count buffers alternate)
    auto count_ge = [&](float thr) -> int {
        int c = 0;
        for (int g = threadIdx.x; g < n; g += nthr) c += v[(size_t)g * stride] >= thr;
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cntb[par][wave] = c;
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += cntb[par][w];
        par ^= 1;
        return tot;
    };
    float lo = lo0, hi = fmaxf(vmax, lo0);
    // when at most K values reach lo0, all of them are taken and no bisection is needed
    if (count_ge(lo0) > K) {
        const int slack = K >> 3;
        for (int it2 = 0; it2 < 40; ++it2) {
            const float mid = 0.5f * (lo + hi);
            if (!(mid > lo && mid < hi)) break;
            const int c = count_ge(mid);
            if (c >= K) {
                lo = mid;
                if (c <= K + slack) break;
            } else {
                hi = mid;
            }
        }
    }
    (void)shf;
    const float thr = lo;
    const int chunk = (n + nthr - 1) / nthr;
    const int g0 = threadIdx.x * chunk, g1 = min(n, g0 + chunk);
    int cnt = 0;
    for (int g = g0; g < g1; ++g) cnt += v[(size_t)g * stride] >= thr;
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
    }
    __syncthreads();
    if (lane == 63) red[wave].i = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < (nthr >> 6); ++w) { const int t0 = red[w].i; red[w].i = acc; acc += t0; }
        shi[2] = acc;
    }
    __syncthreads();
    int pos = red[wave].i + incl - cnt;
    for (int g = g0; g < g1; ++g)
        if (v[(size_t)g * stride] >= thr) {
            if (pos < K) out[pos] = g;
            ++pos;
        }
    __syncthreads();
    return min(K, shi[2]);
}

// A^{-1} = Y[piv]^{-1} (r x r, row stride r) by Gauss-Jordan with partial pivoting: A is held in
// registers (thread t holds row t / 16, columns t % 16 + 16 u, u = 0..3; the maxvol kernels run
// 1024 threads and r <= 64) and A^{-1} in LDS, so that only one r x r matrix occupies LDS; vec
// (LDS, 5 r entries) holds the pivot rows of both, the old row j of both and column j of A.
// An exactly singular pivot leaves its column at zero and sets it.mv_singular (when
// flag_singular). Returns the smallest squared modulus of the pivots (the same in every thread).
constexpr int GJ_THREADS = 1024;
static_assert(GJ_THREADS == 16 * TTFP_MAX_RANK, "one row of A per 16 threads");
__device__ double gj_inverse(const cplx *Y, const int *piv, int r, int m, cplx *Ai, cplx *vec, Item &it,
                             bool flag_singular = true)
{
    cplx *pa = vec, *pi = vec + r, *ja = vec + 2 * r, *ji = vec + 3 * r, *fcol = vec + 4 * r;
    const int a = threadIdx.x >> 4, c0 = threadIdx.x & 15;
    const bool arow = a < r;
    double minp = INFINITY;
    // the thread's four entries of A, in named registers (an array indexed by a runtime slot
    // would be placed in scratch memory)
    cplx ag0 = {0.0, 0.0}, ag1 = {0.0, 0.0}, ag2 = {0.0, 0.0}, ag3 = {0.0, 0.0};
    __syncthreads();
    const cplx *yrow = Y + (size_t)min(max(arow ? piv[a] : 0, 0), m - 1) * r;
    auto init = [&](cplx &v, int c) {
        if (arow && c < r) {
            v = yrow[c];
            Ai[a * r + c] = (a == c) ? cplx{1.0, 0.0} : cplx{0.0, 0.0};
        }
    };
    init(ag0, c0);
    init(ag1, c0 + 16);
    init(ag2, c0 + 32);
    init(ag3, c0 + 48);
    for (int j = 0; j < r; ++j) {
        // column j of A, published by its owners (the threads whose slot u holds column c0 + 16 u = j)
        if (arow) {
            if (c0 == j) fcol[a] = ag0;
            else if (c0 + 16 == j) fcol[a] = ag1;
            else if (c0 + 32 == j) fcol[a] = ag2;
            else if (c0 + 48 == j) fcol[a] = ag3;
        }
        __syncthreads();
        // partial pivoting: the first row of the largest modulus in column j (rows j..r-1), found
        // by every thread from the r - j entries (broadcast LDS reads)
        int p = r;
        double best = -2.0;
        for (int q = j; q < r; ++q) {
            double v = cabs2(fcol[q]);
            if (!(v >= 0.0)) v = -1.0;                  // a non-finite entry ranks below every number
            if (v > best) { best = v; p = q; }
        }
        p = min(p, r - 1);
        const cplx gjj = fcol[p];
        const bool sing = !(fmax(fabs(gjj.x), fabs(gjj.y)) > 0.0) || !(cabs2(gjj) <= 1e300);
        minp = sing ? 0.0 : fmin(minp, cabs2(gjj));
        const cplx inv = sing ? cplx{0.0, 0.0} : cdiv({1.0, 0.0}, gjj);
        if (sing && flag_singular && threadIdx.x == 0) it.mv_singular = 1;
        // rows j and p trade places and the pivot row is scaled: the pivot rows (scaled) and the old
        // rows j of A and of A^{-1}
        auto rows = [&](const cplx &v, int c) {
            if (c < r) {
                if (a == p) {
                    pa[c] = cmul(v, inv);
                    pi[c] = cmul(Ai[p * r + c], inv);
                }
                if (a == j) {
                    ja[c] = v;
                    ji[c] = Ai[j * r + c];
                }
            }
        };
        rows(ag0, c0);
        rows(ag1, c0 + 16);
        rows(ag2, c0 + 32);
        rows(ag3, c0 + 48);
        __syncthreads();
        // elimination; the factor of row a is A(a, j), that of the swapped row p is A(j, j)
        if (arow) {
            const cplx f = a == p ? fcol[j] : fcol[a];
            auto elim = [&](cplx &v, int c) {
                if (c < r) {
                    if (a == j) {
                        v = pa[c];
                        Ai[a * r + c] = pi[c];
                    } else {
                        const cplx ga = a == p ? ja[c] : v, ia = a == p ? ji[c] : Ai[a * r + c];
                        v = csub(ga, cmul(f, pa[c]));
                        Ai[a * r + c] = csub(ia, cmul(f, pi[c]));
                    }
                }
            };
            elim(ag0, c0);
            elim(ag1, c0 + 16);
            elim(ag2, c0 + 32);
            elim(ag3, c0 + 48);
        }
        __syncthreads();
    }
    return minp;
}

// Bc = Y[cand] A^{-1} (Kc x r, row-major) on the FP64 matrix cores: each wave forms 16 x 16 tiles
// of the candidate block one at a time (three real products per complex one, Gauss), so that the
// accumulators take 24 registers and the maxvol kernels keep two workgroups per CU; A^{-1} is in
// LDS with row stride r. Operand and accumulator lane layouts as in k_interp. Every thread of the
// workgroup calls it; control flow is uniform within a wave.
__device__ void block_times_inverse(const cplx *Y, const int *cand, int Kc, int r, const cplx *Ai, cplx *Bc)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4, ntile = (r + 15) / 16;
    const int ntot = ((Kc + 15) / 16) * ntile;
    for (int tt = wave; tt < ntot; tt += nw) {
        const int g0 = 16 * (tt / ntile), q = tt % ntile;
        double4_t prr = {0.0, 0.0, 0.0, 0.0}, pii = {0.0, 0.0, 0.0, 0.0}, pss = {0.0, 0.0, 0.0, 0.0};
        const int arow = g0 + li, jj = 16 * q + li;
        const cplx *y = Y + (size_t)cand[min(arow, Kc - 1)] * r;
        for (int k0 = 0; k0 < r; k0 += 4) {
            const int kk = k0 + lk;
            const cplx a = (arow < Kc && kk < r) ? gld(y + kk) : cplx{0.0, 0.0};
            const cplx b = (kk < r && jj < r) ? Ai[kk * r + jj] : cplx{0.0, 0.0};
            prr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, prr, 0, 0, 0);
            pii = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, pii, 0, 0, 0);
            pss = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, pss, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = g0 + lk + 4 * v;
            if (row < Kc && jj < r) gst(Bc + (size_t)row * r + jj, cplx{prr[v] - pii[v], pss[v] - prr[v] - pii[v]});
        }
    }
}

// maxvol swaps on the candidate block Bc (Kc x r, global memory, rows cand[0..Kc)); returns the
// number of swaps (same in every thread). A swap that puts candidate row q in place of pivot js
// changes one row of A = Y[piv]: B = Y A^{-1} and, when Ai is given (r x r, LDS), A^{-1} itself
// take the same rank-one update (Sherman-Morrison: A'^{-1} = A^{-1} - A^{-1} e_js (B_q - e_js) / B_q,js).
constexpr int MV_SM_MAX = 32;                   // more swaps than this: a fresh Gauss-Jordan inverse
__device__ int swap_block(cplx *Bc, int Kc, int r, const int *cand, int *piv, double lim, int maxit, cplx *prow, cplx *colv,
                          ArgMax *red, cplx *Ai = nullptr, cplx *acol = nullptr)
{
    const int nthr = blockDim.x;
    int swaps = 0;
    const long long tot = (long long)Kc * r;
    // the entry of largest modulus; after each swap it is found in the update pass itself
    ArgMax a = {-1.0, 0x7fffffff};
    for (long long e = threadIdx.x; e < tot; e += nthr) {
        const double v = cabs2(gld(Bc + e));
        a = better(a, ArgMax{v <= 1e300 ? v : -1.0, (int)e});
    }
    a = block_argmax(a, red);
    while (swaps < maxit) {
        if (!(a.v > lim) || a.i < 0 || a.i >= tot) break;
        const int qs = a.i / r, js = a.i % r;
        const cplx b = gld(Bc + (size_t)qs * r + js);
        for (int c = threadIdx.x; c < r; c += nthr) {
            cplx w = gld(Bc + (size_t)qs * r + c);
            if (c == js) w.x -= 1.0;
            prow[c] = w;
        }
        for (int q = threadIdx.x; q < Kc; q += nthr) colv[q] = cdiv(gld(Bc + (size_t)q * r + js), b);
        if (Ai)
            for (int i = threadIdx.x; i < r; i += nthr) acol[i] = cdiv(Ai[i * r + js], b);
        if (threadIdx.x == 0) piv[js] = cand[qs];
        __syncthreads();
        ArgMax an = {-1.0, 0x7fffffff};
        for (long long e = threadIdx.x; e < tot; e += nthr) {
            const int q = (int)(e / r), c = (int)(e % r);
            const cplx v = csub(gld(Bc + e), cmul(colv[q], prow[c]));
            gst(Bc + e, v);
            const double v2 = cabs2(v);
            an = better(an, ArgMax{v2 <= 1e300 ? v2 : -1.0, (int)e});
        }
        if (Ai)
            for (int e = threadIdx.x; e < r * r; e += nthr) Ai[e] = csub(Ai[e], cmul(acol[e / r], prow[e % r]));
        a = block_argmax(an, red);             // its barriers also publish the updated block
        ++swaps;
    }
    __syncthreads();
    return swaps;
}

// Start of maxvol by Gaussian elimination with partial pivoting on a block S (n x r, global
// memory, row g of S is row rowmap[g] of Y, or row g when rowmap is null). chosen[n] flags the
// rows taken (cleared by the caller); gsel (optional) receives the block row of each pivot. Stops
// at the first column whose largest remaining entry has squared modulus <= ptol2 and returns its
// index; returns r when all r pivots were found. A pivot row keeps its values from the step that
// chose it (its entries from that column on are the elimination's U row).
__device__ __forceinline__ int lu_start(cplx *S, int n, int r, const int *rowmap, int *chosen, int *piv, double ptol2, cplx *prow,
                        ArgMax *red, int *shi, int *gsel = nullptr)
{
    const int nthr = blockDim.x;
    for (int j = 0; j < r; ++j) {
        ArgMax a = {-1.0, 0x7fffffff};
        for (int g = threadIdx.x; g < n; g += nthr)
            if (!chosen[g]) {
                const double v = cabs2(S[(size_t)g * r + j]);
                a = better(a, ArgMax{v <= 1e300 ? v : -1.0, g});
            }
        a = block_argmax(a, red);
        if (!(a.v > ptol2) || a.i < 0 || a.i >= n) return j;      // same decision in every thread
        const int p = a.i;
        const cplx pinv = cdiv({1.0, 0.0}, S[(size_t)p * r + j]);
        for (int c = j + 1 + threadIdx.x; c < r; c += nthr) prow[c] = cmul(S[(size_t)p * r + c], pinv);
        if (threadIdx.x == 0) {
            chosen[p] = 1;
            piv[j] = rowmap ? rowmap[p] : p;
            if (gsel) gsel[j] = p;
        }
        __syncthreads();
        const int w = r - j - 1;
        if (w > 0)
            for (long long e = threadIdx.x; e < (long long)n * w; e += nthr) {
                const int g = (int)(e / w), c = j + 1 + (int)(e % w);
                if (chosen[g]) continue;
                S[(size_t)g * r + c] = csub(S[(size_t)g * r + c], cmul(S[(size_t)g * r + j], prow[c]));
            }
        __syncthreads();
    }
    return r;
}

// The same elimination (the same pivots up to rounding) blocked by panels of MV_NB columns: the
// panel of the block's rows is factored in LDS (P, column-major, n x w), then the trailing
// columns of the non-chosen rows take the whole panel's update in one pass over S, with the
// pivot rows' trailing parts V (w x nt, LDS) formed by forward substitution. S is then read and
// written once per panel instead of once per column. Returns r, or the first column without a
// pivot above ptol2 (S is then not in the unblocked elimination's state: the caller eliminates
// again with lu_start). Every thread of the workgroup calls it.
constexpr int MV_NB = 7;
__device__ int lu_start_blocked(cplx *S, int n, int r, const int *rowmap, int *chosen, int *piv, int *gsel, double ptol2,
                                cplx *P, cplx *V, cplx *prow, cplx *pvt, int *pv, ArgMax *red)
{
    const int nthr = blockDim.x;
    for (int j0 = 0; j0 < r; j0 += MV_NB) {
        const int w = min(MV_NB, r - j0);
        for (int e = threadIdx.x; e < n * w; e += nthr) {
            const int g = e / w, t = e % w;
            P[t * n + g] = S[(size_t)g * r + j0 + t];
        }
        __syncthreads();
        for (int t = 0; t < w; ++t) {
            ArgMax a = {-1.0, 0x7fffffff};
            for (int g = threadIdx.x; g < n; g += nthr)
                if (!chosen[g]) {
                    const double v = cabs2(P[t * n + g]);
                    a = better(a, ArgMax{v <= 1e300 ? v : -1.0, g});
                }
            a = block_argmax(a, red);
            if (!(a.v > ptol2) || a.i < 0 || a.i >= n) return j0 + t;     // same decision in every thread
            const int p = a.i;
            const cplx pinv = cdiv({1.0, 0.0}, P[t * n + p]);
            for (int c = t + 1 + threadIdx.x; c < w; c += nthr) prow[c] = cmul(P[c * n + p], pinv);
            if (threadIdx.x == 0) {
                chosen[p] = 1;
                piv[j0 + t] = rowmap ? rowmap[p] : p;
                gsel[j0 + t] = p;
                pv[t] = p;
                pvt[t] = P[t * n + p];
            }
            __syncthreads();
            const int ww = w - t - 1;
            for (int e = threadIdx.x; e < n * ww; e += nthr) {
                const int g = e % n, c = t + 1 + e / n;
                if (!chosen[g]) P[c * n + g] = csub(P[c * n + g], cmul(P[t * n + g], prow[c]));
            }
            __syncthreads();
        }
        const int nt = r - j0 - w;
        if (nt <= 0) break;
        // V[t] = the pivot row p_t's trailing part after the panel's earlier steps, scaled by its pivot
        for (int c = threadIdx.x; c < nt; c += nthr)
            for (int t = 0; t < w; ++t) {
                cplx acc = S[(size_t)pv[t] * r + j0 + w + c];
                for (int t2 = 0; t2 < t; ++t2) acc = csub(acc, cmul(P[t2 * n + pv[t]], V[t2 * nt + c]));
                V[t * nt + c] = cdiv(acc, pvt[t]);
            }
        __syncthreads();
        for (long long e = threadIdx.x; e < (long long)n * nt; e += nthr) {
            const int g = (int)(e / nt), c = (int)(e % nt);
            if (chosen[g]) continue;
            cplx acc = S[(size_t)g * r + j0 + w + c];
            for (int t = 0; t < w; ++t) acc = csub(acc, cmul(P[t * n + g], V[t * nt + c]));
            S[(size_t)g * r + j0 + w + c] = acc;
        }
        __syncthreads();
    }
    return r;
}

// Warm start of a step from the pivots that the previous half sweep in the same direction chose at
// this core: each of its multi-indices (the old index set I_{k+1} of a left-to-right step, J_k of a
// right-to-left one) whose prefix (suffix) is still in the current neighbouring set I_k (J_{k+1})
// names one fiber row, a N + i (i nb + b). Writes those rows to piv and returns their number (the
// same in every thread); returns 0 when two would coincide. Every thread must call it.
__device__ int map_previous_pivots(const Item &it, const StepShape &s, int dir, int *piv, int *shi)
{
    __shared__ int found[TTFP_MAX_RANK];
    const int d = it.d, R = it.R, N = it.N, k = s.k, nthr = blockDim.x;
    const int n_old = min(dir == 0 ? it.nI[k + 1] : it.nJ[k], TTFP_MAX_RANK);
    const int n_cur = dir == 0 ? it.nI[k] : it.nJ[k + 1];
    const int *oldset = it.Iset + (size_t)(k + 1) * R * d, *curset = it.Iset + (size_t)k * R * d;
    if (dir != 0) {
        oldset = it.Jset + (size_t)k * R * d;
        curset = it.Jset + (size_t)(k + 1) * R * d;
    }
    const int c0 = dir == 0 ? 0 : k + 1, c1 = dir == 0 ? k : d;     // the shared coordinates
    __syncthreads();
    for (int q = threadIdx.x; q < n_old; q += nthr) found[q] = -1;
    __syncthreads();
    for (int e = threadIdx.x; e < n_old * n_cur; e += nthr) {
        const int q = e / n_cur, a = e % n_cur;
        bool match = true;
        for (int c = c0; c < c1 && match; ++c) match = oldset[q * d + c] == curset[a * d + c];
        if (match) found[q] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int n0 = 0;
        for (int q = 0; q < n_old; ++q) {
            const int a = found[q];
            if (a < 0) continue;
            const int i = oldset[q * d + k];
            if (i < 0 || i >= N) continue;
            const int row = dir == 0 ? a * N + i : i * n_cur + a;
            if (row < 0 || row >= s.rows) continue;
            bool dup = false;
            for (int u = 0; u < n0 && !dup; ++u) dup = piv[u] == row;
            if (dup) { n0 = 0; break; }
            piv[n0++] = row;
        }
        shi[3] = n0;
    }
    __syncthreads();
    return shi[3];
}

// The largest squared column norm of A^{-1} (LDS, r x r, row stride r), by wave 0, into
// it.mv_colmax: with the squared row norms of Y it bounds every |B_ij|^2 = |y_i A^{-1} e_j|^2 by
// Cauchy-Schwarz, which lets k_interp's checking passes skip rows that cannot violate.
__device__ void store_colmax(const cplx *Ai, int r, Item &it)
{
    if (threadIdx.x < 64) {
        double v = 0.0;
        if ((int)threadIdx.x < r)
            for (int k = 0; k < r; ++k) v += cabs2(Ai[k * r + threadIdx.x]);
        v = wave_max(v);
        if (threadIdx.x == 0) it.mv_colmax = v;
    }
}

// Abuf is dynamic LDS of max(rmax^2, 8 MV_KMAX) complex entries (64 KiB; rmax: the largest rank
// of the launch): the key buffer of the start, the blocked elimination's panel, then A^{-1} (the
// Gauss-Jordan inverse keeps A itself in registers). With the static arrays a workgroup takes
// under 80 KiB, so two run on a CU. 1024 threads.
__global__ __launch_bounds__(1024, 8) void k_maxvol(Item *items, ItemList work, int t, int dir, int rmax, int warm)
{
    extern __shared__ cplx Abuf[];
    const int cap = max(rmax * rmax, MV_KMAX * (MV_NB + 1));   // entries of Abuf
    cplx *Ai = Abuf;
    __shared__ cplx prow[TTFP_MAX_RANK];
    __shared__ cplx fcol[TTFP_MAX_RANK];
    __shared__ int piv[TTFP_MAX_RANK];
    __shared__ int gsel[TTFP_MAX_RANK];
    __shared__ cplx pvt[MV_NB];
    __shared__ int pv[MV_NB];
    __shared__ int cand[MV_KMAX];
    __shared__ cplx colv[MV_KMAX];
    int *chosen = reinterpret_cast<int *>(colv);     // the start's row flags (colv is free then)
    __shared__ ArgMax red[17];
    __shared__ int shi[4];
    __shared__ float shf[2];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int m = s.rows, r = it.rsel;
    const cplx *Y = it.Y;
    cplx *W = it.W;
    cplx *B = (dir != 2) ? it.cores + (size_t)s.k * it.R * it.N * it.R : it.Bt;
    const int nthr = blockDim.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // ---- 1a. row norms (one key per group of gsz consecutive rows: its largest norm); the
    // violation marks that k_interp records are cleared
    const int nkeys = cap * (int)(sizeof(cplx) / sizeof(float));
    const int gsz = (m + nkeys - 1) / nkeys;            // 1 unless m exceeds the key buffer
    const int nk = (m + gsz - 1) / gsz;
    // the start's candidate block: the MV_KMAX rows of largest leverage (a larger block gives a
    // start nearer to dominant and fewer swaps and refinement rounds after it: 79.3 options/s on
    // the d = 5 headline batch of 192 options against 75.3 with max(4 r, 64) rows, one box)
    int K = MV_KMAX;
    K = min(K, nk);
    float *key = (float *)Abuf;
    float kmax = 0.0f;
    for (int g = threadIdx.x; g < nk; g += nthr) {
        float best = -1.0f;
        for (int i = g * gsz; i < min(m, (g + 1) * gsz); ++i) {
            float q;
            if (dir != 2) {
                q = it.keys[i];                          // the row norm written by k_basis
            } else {
                const cplx *y = Y + (size_t)i * r;
                double qq = 0.0;
                for (int c = 0; c < r; ++c) qq += cabs2(y[c]);
                q = (float)qq;
            }
            it.viol[i] = 0.0f;
            if (!(q >= 0.0f && q <= 3.0e38f)) q = 0.0f;     // a non-finite row is never a pivot
            best = fmaxf(best, q);
        }
        key[g] = fmaxf(best, 0.0f);
        kmax = fmaxf(kmax, key[g]);
    }
    {
        ArgMax a = {(double)kmax, 0};
        a = block_argmax(a, red);
        kmax = (float)a.v;
    }
    // ---- 1b. the K largest groups, resolved to their largest-norm row
    const int Kc = select_largest(key, 1, nk, K, 0.0f, kmax, cand, red, shi, shf);
    for (int q = threadIdx.x; q < Kc; q += nthr) {
        const int g = cand[q];
        int bi = g * gsz;
        double best = -1.0;
        for (int i = g * gsz; i < min(m, (g + 1) * gsz); ++i) {
            const cplx *y = Y + (size_t)i * r;
            double v = 0.0;
            for (int c = 0; c < r; ++c) v += cabs2(y[c]);
            if (v > best) { best = v; bi = i; }
        }
        cand[q] = bi;
    }
    __syncthreads();
    // ---- 1c. start: elimination with partial pivoting on the block S = Y[cand] (a copy in W).
    // A pivot below 1e-6 of the largest row norm means the block is numerically rank deficient
    // (this happens when many integrand values underflow to zero and the largest rows share
    // their support); the start is then taken on the 2048 largest rows, and failing that on
    // all m rows (row flags and the larger block's row list live in the output B, which only
    // k_interp writes).
    const double ptol2 = 1e-12 * (double)kmax;
    // Warm start (warm = 1, from the second half sweep in a direction on): the pivots of the
    // previous half sweep in this direction, when all r of them name rows of this fiber and their
    // block is not near-singular (smallest Gauss-Jordan pivot above the elimination's threshold);
    // the elimination start is then skipped and A^{-1} is already formed.
    bool warm_ok = false;
    if (warm && dir != 2 && it.half >= 2 + dir && map_previous_pivots(it, s, dir, piv, shi) == r)
        warm_ok = gj_inverse(Y, piv, r, m, Ai, colv, it, false) > ptol2;
    if (!warm_ok) {
        cplx *S = W;
        for (long long e = threadIdx.x; e < (long long)Kc * r; e += nthr)
            S[e] = Y[(size_t)cand[e / r] * r + e % r];
        for (int g = threadIdx.x; g < Kc; g += nthr) chosen[g] = 0;
        __syncthreads();
        // panel-blocked in LDS (the panel in Abuf, the pivot rows' trailing parts after it)
        int nf = lu_start_blocked(S, Kc, r, cand, chosen, piv, gsel, ptol2, Abuf, Abuf + MV_KMAX * MV_NB, prow, pvt, pv, red);
        if (nf < r) {
            // a rank-deficient block: eliminated again unblocked, which leaves the pivot rows as
            // the continuation below needs them
            for (long long e = threadIdx.x; e < (long long)Kc * r; e += nthr)
                S[e] = Y[(size_t)cand[e / r] * r + e % r];
            for (int g = threadIdx.x; g < Kc; g += nthr) chosen[g] = 0;
            __syncthreads();
            nf = lu_start(S, Kc, r, cand, chosen, piv, ptol2, prow, red, shi, gsel);
        }
        if (nf < r) {
            // The block spans only nf dimensions (this happens when many integrand values underflow
            // to zero and the largest rows share their support): the elimination continues over all
            // m rows. With U the nf pivot rows as eliminated (U11 their leading triangle, U12 the
            // rest), every row's residual in the columns nf..r-1 is R_i = Y[i, nf:] - Y[i, :nf] T,
            // T = U11^{-1} U12 (the values the same elimination would leave in it); elimination
            // with partial pivoting on R gives the remaining pivots.
            const int w = r - nf;
            int *flag = reinterpret_cast<int *>(B);      // m row flags (B is written only by k_interp)
            cplx *U = Abuf;                              // nf x r (nf r < cap)
            for (int e = threadIdx.x; e < nf * r; e += nthr) U[e] = S[(size_t)gsel[e / r] * r + e % r];
            for (int i = threadIdx.x; i < m; i += nthr) flag[i] = 0;
            __syncthreads();
            for (int q = threadIdx.x; q < nf; q += nthr) flag[piv[q]] = 1;
            // T in place of U12 by back substitution, one column per thread
            for (int c = threadIdx.x; c < w; c += nthr)
                for (int q = nf - 1; q >= 0; --q) {
                    cplx acc = U[q * r + nf + c];
                    for (int q2 = q + 1; q2 < nf; ++q2) acc = csub(acc, cmul(U[q * r + q2], U[q2 * r + nf + c]));
                    U[q * r + nf + c] = cdiv(acc, U[q * r + q]);
                }
            __syncthreads();
            cplx *Rm = W;                                // m x w residuals (the block copy is no longer needed)
            for (long long e = threadIdx.x; e < (long long)m * w; e += nthr) {
                const int i = (int)(e / w), c = (int)(e % w);
                const cplx *y = Y + (size_t)i * r;
                cplx acc = y[nf + c];
                for (int q = 0; q < nf; ++q) acc = csub(acc, cmul(y[q], U[q * r + nf + c]));
                Rm[e] = acc;
            }
            __syncthreads();
            nf += lu_start(Rm, m, w, nullptr, flag, piv + nf, 0.0, prow, red, shi);
            if (nf < r) {
                // Y itself is rank deficient: the remaining pivots are the lowest untaken rows
                if (threadIdx.x == 0) {
                    int next = 0;
                    for (int j = nf; j < r; ++j) {
                        bool used = true;
                        while (used && next < m) {
                            used = false;
                            for (int q = 0; q < j; ++q) used |= piv[q] == next;
                            if (used) ++next;
                        }
                        piv[j] = min(next, m - 1);
                        ++next;
                    }
                    it.mv_singular = 1;
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) it.mv_full += 1;
        }
        __syncthreads();
        // ---- 2. A^{-1} (unless the warm start formed it)
        gj_inverse(Y, piv, r, m, Ai, colv, it);
    }
    // the block's rows of B (in W, over the start's copy)
    cplx *Bc = W;
    block_times_inverse(Y, cand, Kc, r, Ai, Bc);
    __syncthreads();
    // ---- 3. swaps within the block, 4. A^{-1} of the final pivots
    const double lim = (1.0 + it.delta) * (1.0 + it.delta);
    const int swaps = swap_block(Bc, Kc, r, cand, piv, lim, 4 * r + 16, prow, colv, red, Ai, fcol);
    if (swaps > MV_SM_MAX) gj_inverse(Y, piv, r, m, Ai, colv, it);
    __syncthreads();
    for (int e = threadIdx.x; e < r * r; e += nthr) it.Ai[e] = Ai[e];
    for (int c = threadIdx.x; c < r; c += nthr) it.piv[c] = piv[c];
    store_colmax(Ai, r, it);
    if (threadIdx.x == 0) {
        it.mv_iters += swaps;
        it.mv_viol = 0;
        it.mv_dirty = 1;
        // Bc (8 Kc r^2), one rank-one update of Bc and A^{-1} per swap (8 (Kc + r) r),
        // Gauss-Jordan (8 r^3 each)
        it.work[TTFP_KERNEL_MAXVOL] += 8.0 * Kc * (double)r * r + 8.0 * (Kc + r) * (double)r * swaps +
                                       8.0 * (double)r * r * r * (swaps > MV_SM_MAX ? 2 : 1);
    }
}

// Refinement round: the pivots and up to MV_KMAX - r rows that k_interp found violating (largest
// first) form the block; swaps as in k_maxvol. Returns at once when no row violated.
__global__ __launch_bounds__(1024, 8) void k_maxvol_refine(Item *items, ItemList work, int t, int dir, int rmax, int *moved)
{
    extern __shared__ cplx Abuf[];
    cplx *Ai = Abuf;                                 // rmax^2 entries
    __shared__ cplx prow[TTFP_MAX_RANK];
    __shared__ cplx fcol[TTFP_MAX_RANK];
    __shared__ int piv[TTFP_MAX_RANK];
    __shared__ int cand[MV_KMAX];
    __shared__ cplx colv[MV_KMAX];
    __shared__ ArgMax red[17];
    __shared__ int shi[4];
    __shared__ float shf[2];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    if (!it.mv_viol) {
        if (threadIdx.x == 0) it.mv_dirty = 0;
        return;
    }
    const int m = s.rows, r = it.rsel, nthr = blockDim.x;
    const cplx *Y = it.Y;
    cplx *W = it.W;
    for (int c = threadIdx.x; c < r; c += nthr) {
        piv[c] = it.piv[c];
        cand[c] = piv[c];
    }
    float vmax = 0.0f;
    for (int i = threadIdx.x; i < m; i += nthr) vmax = fmaxf(vmax, it.viol[i]);
    {
        ArgMax a = {(double)vmax, 0};
        a = block_argmax(a, red);
        vmax = (float)a.v;
    }
    // the pivots and up to MV_KMAX - r of the worst violators (a larger block than the start's:
    // more swaps per round, so fewer rounds reach the same dominance)
    const int K = min(MV_KMAX, m);
    // only rows that violated (a positive mark) are candidates
    const int nv = select_largest(it.viol, 1, m, K - r, 1e-30f, vmax, cand + r, red, shi, shf);
    const int Kc = r + nv;
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += nthr) it.viol[i] = 0.0f;   // for the next k_interp
    // block rows: the pivots (rows of the identity) and the violating rows of B = Y A^{-1},
    // formed here on the matrix cores (the checking passes of k_interp do not store B)
    cplx *Bc = W;
    for (int e = threadIdx.x; e < r * r; e += nthr) {
        Ai[e] = it.Ai[e];
        Bc[e] = cplx{e / r == e % r ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    block_times_inverse(Y, cand + r, Kc - r, r, Ai, Bc + (size_t)r * r);
    __syncthreads();
    const double lim = (1.0 + it.delta) * (1.0 + it.delta);
    const int swaps = swap_block(Bc, Kc, r, cand, piv, lim, 4 * r + 16, prow, colv, red, Ai, fcol);
    if (swaps > MV_SM_MAX) gj_inverse(Y, piv, r, m, Ai, colv, it);
    __syncthreads();
    if (swaps > 0) {
        for (int e = threadIdx.x; e < r * r; e += nthr) it.Ai[e] = Ai[e];
        for (int c = threadIdx.x; c < r; c += nthr) it.piv[c] = piv[c];
        store_colmax(Ai, r, it);
    }
    if (threadIdx.x == 0) {
        it.mv_iters += swaps;
        it.mv_viol = 0;
        it.mv_dirty = swaps > 0;
        if (swaps > 0 && moved) moved[1 + atomicAdd(moved, 1)] = item;
        it.work[TTFP_KERNEL_REFINE] += 8.0 * (Kc + r) * (double)r * swaps + (swaps > MV_SM_MAX ? 8.0 * (double)r * r * r : 0.0);
    }
}

// Empties the list of items whose pivots moved (its length in moved[0]) before a refinement round.
__global__ void k_clear_moved(int *moved)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) moved[0] = 0;
}

// B = Y A^{-1} for every row on the FP64 matrix cores: a wave forms a 16-row panel of B (all r
// columns, as up to four 16 x 16 tiles) with v_mfma_f64_16x16x4f64, the complex product as three
// real ones (Gauss: re = Yr Ar - Yi Ai, im = (Yr + Yi)(Ar + Ai) - Yr Ar - Yi Ai; the rounding
// error stays of the order of |Y||A| as with four products); A^{-1} is held in LDS. Lane l supplies
// A-operand entry (row l % 16, k l / 16) and B-operand entry (k l / 16, column l % 16), and holds
// accumulator rows l / 16 + 4 v, column l % 16 (v = 0..3; the layout was checked by a probe
// against a host product). B goes straight into the core's slot. Rows whose largest |B_ij|
// exceeds 1 + delta are marked (largest squared modulus in viol) and the item is flagged for a
// refinement round. mode 0: a checking pass over every item; mode 1: a checking pass, only after a
// refinement that moved a pivot; mode 2: the final pass over every item, which stores B (into the
// core slot) and marks nothing. Only the final pass writes B: a checking pass reads Y and writes
// the marks alone.
// INTERP_WAVES waves per workgroup, PPW 16-row panels per wave, as for k_basis.
template <int INTERP_WAVES, int PPW>
__global__ __launch_bounds__(64 * INTERP_WAVES, 4) void k_interp(Item *items, ItemList work, int t, int dir, int mode, int bound)
{
    __shared__ cplx Ai[TTFP_MAX_RANK * TTFP_MAX_RANK];
    // a checking pass over the items whose pivots moved (a list with a device-side length) runs in
    // block-major order, so that the blocks past the list's length come at the end of the launch
    const bool moved_list = work.count != nullptr;
    const int item = work.item(moved_list ? blockIdx.y : blockIdx.x), wblk = moved_list ? blockIdx.x : blockIdx.y;
    if (item < 0 || !work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    if (mode == 1 && !it.mv_dirty) return;
    const bool store = mode == 2;
    const int r = it.rsel, m = s.rows;
    const int rows_per_wg = 16 * INTERP_WAVES * PPW;
    if (wblk * rows_per_wg >= m) return;
    const double lim = (1.0 + it.delta) * (1.0 + it.delta);
    // A checking pass skips the rows that cannot violate: |B_ij|^2 <= |y_i|^2 max_j |A^{-1} e_j|^2
    // (the row norms from k_basis, held as floats: the margin covers their rounding). A workgroup
    // whose rows all stay below the bound returns before staging A^{-1}; so does a wave.
    const bool check = !store && dir != 2 && bound;
    const double cm = 1.001 * it.mv_colmax;
    if (check) {
        const int row = wblk * rows_per_wg + (int)threadIdx.x;
        const bool need = (int)threadIdx.x < rows_per_wg && row < m && !((double)gld(it.keys + row) * cm <= lim);
        if (!__syncthreads_or(need)) return;
    }
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) Ai[e] = it.Ai[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
    for (int pp = 0; pp < PPW; ++pp) {
        const int row0 = wblk * rows_per_wg + (pp * INTERP_WAVES + wave) * 16;
        if (row0 >= m) break;
        const int li = lane & 15, lk = lane >> 4;
        if (check) {
            const int row = row0 + li;
            if (!__any(row < m && !((double)gld(it.keys + row) * cm <= lim))) continue;
        }
        // the work done: this panel's rows
        if (lane == 0) atomicAdd(&it.work[TTFP_KERNEL_INTERP], 8.0 * (double)min(16, m - row0) * r * r);
        const int ntile = (r + 15) / 16;
        const cplx *Y = it.Y;
        // complex products by three real ones (Gauss): prr = Ar Br, pii = Ai Bi, pss = (Ar + Ai)(Br + Bi);
        // re = prr - pii, im = pss - prr - pii
        double4_t prr[4], pii[4], pss[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            prr[q] = double4_t{0.0, 0.0, 0.0, 0.0};
            pii[q] = double4_t{0.0, 0.0, 0.0, 0.0};
            pss[q] = double4_t{0.0, 0.0, 0.0, 0.0};
        }
        const int arow = row0 + li;
        // the left operand of the next k-step is loaded while this one's products run
        cplx an = (arow < m && lk < r) ? gld(Y + (size_t)arow * r + lk) : cplx{0.0, 0.0};
        for (int k0 = 0; k0 < r; k0 += 4) {
            const int kk = k0 + lk;
            const cplx a = an;
            if (k0 + 4 < r) an = (arow < m && kk + 4 < r) ? gld(Y + (size_t)arow * r + kk + 4) : cplx{0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= ntile) break;
                const int jj = 16 * q + li;
                const cplx b = (kk < r && jj < r) ? Ai[kk * r + jj] : cplx{0.0, 0.0};
                prr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, prr[q], 0, 0, 0);
                pii[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, pii[q], 0, 0, 0);
                pss[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, pss[q], 0, 0, 0);
            }
        }
        // the core slot holds B itself for a left-to-right step (rows (a, i), columns b: the core's
        // a x N x b layout) and B transposed for a right-to-left one (rows (i, b), columns a);
        // the raw entry point's B is row-major in Bt
        cplx *B = (dir != 2) ? it.cores + (size_t)s.k * it.R * it.N * it.R : it.Bt;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + lk + 4 * v;
            double mx = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q >= ntile) break;
                const int col = 16 * q + li;
                if (row < m && col < r) {
                    const cplx val = {prr[q][v] - pii[q][v], pss[q][v] - prr[q][v] - pii[q][v]};
                    if (store) gst(B + (dir == 1 ? (size_t)col * m + row : (size_t)row * r + col), val);
                    mx = fmax(mx, cabs2(val));
                }
            }
            if (store) continue;
            // largest entry of the row over the 16 lanes that hold its columns
            for (int o = 8; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
            if (li == 0 && row < m && mx > lim && mx <= 1e300) {
                atomicMax(reinterpret_cast<unsigned int *>(it.viol + row), __float_as_uint((float)mx));
                it.mv_viol = 1;
            }
        }
    }
}
template __global__ void k_interp<8, 1>(Item *, ItemList, int, int, int, int);
template __global__ void k_interp<16, 1>(Item *, ItemList, int, int, int, int);
template __global__ void k_interp<8, 2>(Item *, ItemList, int, int, int, int);
template __global__ void k_interp<16, 2>(Item *, ItemList, int, int, int, int);

// ------------------------------------------------------------------ index sets and core placement
__global__ __launch_bounds__(256) void k_finish(Item *items, ItemList work, int t, int dir)
{
    const int item = work.item(blockIdx.y);
    if (!work.active[item]) return;
    Item &it = items[item];
    StepShape s = step_shape(it, t, dir, 0);
    if (!s.valid) return;
    const int r = it.rsel, d = it.d, N = it.N, R = it.R, k = s.k;
    if (dir == 0) {
        const int *Ik = it.Iset + (size_t)k * R * d;
        int *In = it.Iset + (size_t)(k + 1) * R * d;
        for (int q = threadIdx.x; q < r; q += blockDim.x) {
            const int row = min(max(it.piv[q], 0), s.rows - 1), a = row / N, i = row % N;
            for (int c = 0; c < k; ++c) In[q * d + c] = Ik[a * d + c];
            In[q * d + k] = i;
        }
        if (threadIdx.x == 0) {
            it.crow[k] = it.nI[k];
            it.ccol[k] = r;
            it.nI[k + 1] = r;
            it.n_evals += (long long)s.rows * s.nc;
        }
    } else {
        const int nb = it.nJ[k + 1];
        const int *J1 = it.Jset + (size_t)(k + 1) * R * d;
        int *Jn = it.Jset + (size_t)k * R * d;
        for (int q = threadIdx.x; q < r; q += blockDim.x) {
            const int row = min(max(it.piv[q], 0), s.rows - 1), i = row / nb, b = row % nb;
            Jn[q * d + k] = i;
            for (int c = k + 1; c < d; ++c) Jn[q * d + c] = J1[b * d + c];
        }
        if (threadIdx.x == 0) {
            it.crow[k] = r;
            it.ccol[k] = nb;
            it.nJ[k] = r;
            it.n_evals += (long long)s.rows * s.nc;
        }
    }
}

// ------------------------------------------------------------------ core sums and contraction
// M_k = sum_i core_k[:, i, :] (the quadrature weights eta_k are applied on the host).
__global__ __launch_bounds__(256) void k_core_sum(Item *items, ItemList work, int t, int dir, int mode)
{
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    int k;
    if (mode == 0) {
        if (t > it.d - 2) return;
        k = step_core(it, t, dir);
    } else {
        k = dir == 0 ? it.d - 1 : 0;
    }
    const int a_n = it.crow[k], b_n = it.ccol[k], N = it.N, R = it.R;
    const int e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= a_n * b_n) return;
    const int a = e / b_n, b = e % b_n;
    const cplx *col = it.cores + (size_t)k * R * N * R + (size_t)a * N * b_n + b;
    // the sum runs over i in order; the loads are issued eight at a time ahead of the additions
    cplx acc = {0.0, 0.0};
    int i = 0;
    for (; i + 8 <= N; i += 8) {
        cplx v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = gld(col + (size_t)(i + u) * b_n);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
    for (; i < N; ++i) acc = cadd(acc, gld(col + (size_t)i * b_n));
    it.M[(size_t)k * R * R + e] = acc;
}

// P = 1^T M_0 M_1 ... M_{d-1} 1
__global__ __launch_bounds__(64) void k_contract(Item *items, ItemList work)
{
    __shared__ cplx v[TTFP_MAX_RANK], w[TTFP_MAX_RANK];
    const int item = work.item(blockIdx.x);
    if (!work.active[item]) return;
    Item &it = items[item];
    if (threadIdx.x == 0) v[0] = {1.0, 0.0};
    __syncthreads();
    for (int k = 0; k < it.d; ++k) {
        const int a_n = it.crow[k], b_n = it.ccol[k];
        const cplx *Mk = it.M + (size_t)k * it.R * it.R;
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
            cplx acc = {0.0, 0.0};
            for (int a = 0; a < a_n; ++a) acc = cadd(acc, cmul(v[a], Mk[a * b_n + b]));
            w[b] = acc;
        }
        __syncthreads();
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) v[b] = w[b];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        it.P = v[0];
        it.half += 1;
    }
}

// ------------------------------------------------------------------ ladders: one cross, many market points
// W[s][i] = exp(-i z_k(i) dm[s][k]) for core k of the item, z_k(i) = u_k(i) + i alpha_k: the factor
// by which point s's integrand differs from the base option's along coordinate k (the mean of w
// shifted by dm[s]).
__global__ __launch_bounds__(256) void k_ladder_weights(const Item *items, int item, int k, int S, const double *dm,
                                                        cplx *W)
{
    const Item &it = items[item];
    const int N = it.N;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)S * N) return;
    const int s = (int)(e / N), i = (int)(e % N);
    const double L = it.L[k];
    const double x = -L + (i + 0.5) * 2.0 * L / N, y = it.alpha[k];
    const double dmv = dm[(size_t)s * it.d + k];
    W[e] = cexp_({y * dmv, -x * dmv});           // -i (x + i y) dm
}

// T[s][a][b] = sum_i W[s][i] G_k[a][i][b]: for each left index a, a points x nodes by nodes x r_k
// product on the FP64 matrix cores (v_mfma_f64_16x16x4f64, lane layout as in k_interp: A-operand
// lane (row l % 16, k l / 16), B-operand lane (k l / 16, column l % 16), accumulator rows
// l / 16 + 4 v). A wave forms 16 points x all r_k columns (up to four 16 x 16 tiles), the complex
// product by three real ones (Gauss). T rows have stride R (T[(s R + a) R + b]).
constexpr int LAD_WAVES = 4;
__global__ __launch_bounds__(64 * LAD_WAVES) void k_ladder_core(const Item *items, int item, int k, int S,
                                                               const cplx *W, cplx *T)
{
    const Item &it = items[item];
    const int N = it.N, R = it.R, a_n = it.crow[k], b_n = it.ccol[k];
    const int a = blockIdx.y;
    if (a >= a_n) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int s0 = (blockIdx.x * LAD_WAVES + wave) * 16;
    if (s0 >= S) return;
    const cplx *G = it.cores + (size_t)k * R * N * R + (size_t)a * N * b_n;   // G[i][b] at i b_n + b
    const int ntile = (b_n + 15) / 16;
    double4_t prr[4], pii[4], pss[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        prr[q] = double4_t{0.0, 0.0, 0.0, 0.0};
        pii[q] = prr[q];
        pss[q] = prr[q];
    }
    const int srow = s0 + li;
    for (int i0 = 0; i0 < N; i0 += 4) {
        const int i = i0 + lk;
        const cplx w = (srow < S && i < N) ? W[(size_t)srow * N + i] : cplx{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= ntile) break;
            const int col = 16 * q + li;
            const cplx g = (i < N && col < b_n) ? G[(size_t)i * b_n + col] : cplx{0.0, 0.0};
            prr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(w.x, g.x, prr[q], 0, 0, 0);
            pii[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(w.y, g.y, pii[q], 0, 0, 0);
            pss[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(w.x + w.y, g.x + g.y, pss[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = s0 + lk + 4 * v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= ntile) break;
            const int col = 16 * q + li;
            if (row < S && col < b_n)
                T[((size_t)row * R + a) * R + col] = {prr[q][v] - pii[q][v], pss[q][v] - prr[q][v] - pii[q][v]};
        }
    }
}

// V[s] <- V[s] T[s] (row vector times r_{k-1} x r_k), one workgroup per point; the chain starts
// from the row vector (1) at the first core.
__global__ __launch_bounds__(64) void k_ladder_chain(const Item *items, int item, int k, int S, const cplx *T, cplx *V)
{
    __shared__ cplx v[TTFP_MAX_RANK];
    const Item &it = items[item];
    const int R = it.R, a_n = it.crow[k], b_n = it.ccol[k], s = blockIdx.x;
    if (s >= S) return;
    for (int a = threadIdx.x; a < a_n; a += blockDim.x) v[a] = k == 0 ? cplx{a == 0 ? 1.0 : 0.0, 0.0} : V[(size_t)s * R + a];
    __syncthreads();
    for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
        cplx acc = {0.0, 0.0};
        for (int a = 0; a < a_n; ++a) acc = cadd(acc, cmul(v[a], T[((size_t)s * R + a) * R + b]));
        V[(size_t)s * R + b] = acc;
    }
}

// ------------------------------------------------------------------ inner product of two tensor trains
// <B|A> = sum_i B(i) A(i) (no conjugation: the integrand is the product of the two functions),
// core by core with the environment E[a1][a2] (a1: B's left index, a2: A's):
//   X[a2][i][b1] = sum_a1 E[a1][a2] B_k[a1][i][b1]          (k_inner_x, one thread per entry)
//   E'[b1][b2]   = sum_{a2, i} X[a2][i][b1] A_k[a2][i][b2]   (k_inner_e, one thread per entry)
// E starts as the 1 x 1 matrix (1); after the last core E[0][0] is the inner product. Cores are laid
// out a x N x b (entry (a N + i) b_n + b of the item's slot k); E has row stride RE.
constexpr int INNER_RE = TTFP_MAX_RANK;
__global__ __launch_bounds__(256) void k_inner_x(const Item *items, int ia, int ib, int k, const cplx *E, cplx *X)
{
    const Item &A = items[ia], &B = items[ib];
    const int N = A.N, a1n = B.crow[k], b1n = B.ccol[k], a2n = A.crow[k];
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)a2n * N * b1n) return;
    const int a2 = (int)(e / ((long long)N * b1n)), rem = (int)(e % ((long long)N * b1n)), i = rem / b1n, b1 = rem % b1n;
    const cplx *Bk = B.cores + (size_t)k * B.R * N * B.R;
    cplx acc = {0.0, 0.0};
    for (int a1 = 0; a1 < a1n; ++a1) {
        const cplx ev = k == 0 ? cplx{1.0, 0.0} : E[a1 * INNER_RE + a2];
        acc = cadd(acc, cmul(ev, Bk[((size_t)a1 * N + i) * b1n + b1]));
    }
    X[e] = acc;
}
__global__ __launch_bounds__(256) void k_inner_e(const Item *items, int ia, int ib, int k, const cplx *X, cplx *E)
{
    const Item &A = items[ia], &B = items[ib];
    const int N = A.N, b1n = B.ccol[k], a2n = A.crow[k], b2n = A.ccol[k];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b1n * b2n) return;
    const int b1 = e / b2n, b2 = e % b2n;
    const cplx *Ak = A.cores + (size_t)k * A.R * N * A.R;
    cplx acc = {0.0, 0.0};
    for (int a2 = 0; a2 < a2n; ++a2)
        for (int i = 0; i < N; ++i)
            acc = cadd(acc, cmul(X[((size_t)a2 * N + i) * b1n + b1], Ak[((size_t)a2 * N + i) * b2n + b2]));
    E[b1 * INNER_RE + b2] = acc;
}

// ------------------------------------------------------------------ convergence test on the device
// After a half sweep: each option's price is the scaled sum of its items' contractions; its
// relative change against the previous half sweep decides whether it stays active (the rule
// of the sweep driver: converged when the change is at most tol after the first half sweep;
// stopped at its last half sweep, or when a rank-capped cross's change no longer halves over a
// full sweep). The items of stopped options are switched off for the kernels that follow.
// flags[c] (c = the launch's half-sweep counter, flags[MAX_HALF]) is set when an option is
// still active, and the host reads it one half sweep later.
__global__ __launch_bounds__(256) void k_converge(const Item *items, int *active, OptState *os, int n_opts,
                                                  const double *item_scale, int *flags)
{
    __shared__ int any;
    const int c = flags[MAX_HALF];
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int o = threadIdx.x; o < n_opts; o += blockDim.x) {
        OptState &st = os[o];
        if (!st.active) continue;
        double pr = 0.0, pi = 0.0;
        int cap = 0;
        for (int i = st.first; i < st.first + st.count; ++i) {
            pr += item_scale[i] * items[i].P.x;
            pi += item_scale[i] * items[i].P.y;
            cap |= items[i].capped;
        }
        const int h = st.half;
        double change = INFINITY;
        if (h > 0) change = fabs(pr - st.prev) / fmax(fabs(pr), 1e-300);
        if (h < 64) st.hist[h] = change;
        const bool last = h == st.max_half - 1;
        const bool stalled = cap && h >= 3 && h < 64 && change > 0.5 * st.hist[h - 2];
        int act = 1;
        if (h >= 1 && change <= st.tol) {
            st.converged = 1;
            act = 0;
        } else if (last || stalled) {
            act = 0;
        }
        st.prev = pr;
        st.price = pr;
        st.imag = pi;
        st.change = change;
        st.capped = cap;
        st.half = h + 1;
        st.active = act;
        if (!act)
            for (int i = st.first; i < st.first + st.count; ++i) active[i] = 0;
        else
            any = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (c < MAX_HALF) flags[c] = any;
        flags[MAX_HALF] = c + 1;
    }
}

// ------------------------------------------------------------------ node moments for the Greeks
// M1_k = sum_i z_k(i) core_k[:, i, :], M2_k = sum_i z_k(i)^2 core_k[:, i, :]
__global__ __launch_bounds__(256) void k_core_moments(Item *items, const int *active)
{
    const int item = blockIdx.z;
    if (!active[item]) return;
    Item &it = items[item];
    const int k = blockIdx.y;
    if (k >= it.d) return;
    const int a_n = it.crow[k], b_n = it.ccol[k], N = it.N, R = it.R;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a_n * b_n) return;
    const int a = e / b_n, b = e % b_n;
    const cplx *core = it.cores + (size_t)k * R * N * R;
    const double L = it.L[k], eta = 2.0 * L / N, al = it.alpha[k];
    cplx s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    for (int i = 0; i < N; ++i) {
        const cplx z = {-L + (i + 0.5) * eta, al};
        const cplx g = core[((size_t)a * N + i) * b_n + b];
        const cplx zg = cmul(z, g);
        s1 = cadd(s1, zg);
        s2 = cadd(s2, cmul(z, zg));
    }
    it.M1[(size_t)k * R * R + e] = s1;
    it.M2[(size_t)k * R * R + e] = s2;
}

// mu1[k] = <TT, z_k>, mu2[k][l] = <TT, z_k z_l> through left/right environments of the chain.
__global__ __launch_bounds__(64) void k_moments(Item *items, const int *active, cplx *out, int stride)
{
    __shared__ cplx lenv[TTFP_MAX_D][TTFP_MAX_RANK];
    __shared__ cplx renv[TTFP_MAX_D][TTFP_MAX_RANK];
    __shared__ cplx v[TTFP_MAX_RANK], w[TTFP_MAX_RANK];
    const int item = blockIdx.x;
    if (!active[item]) return;
    Item &it = items[item];
    const int d = it.d, R = it.R;
    cplx *o = out + (size_t)item * stride;     // [d] mu1 then [d*d] mu2
    // left environments: lenv[k] = 1^T M_0 ... M_{k-1}
    if (threadIdx.x == 0) lenv[0][0] = {1.0, 0.0};
    __syncthreads();
    for (int k = 0; k + 1 < d; ++k) {
        const int a_n = it.crow[k], b_n = it.ccol[k];
        const cplx *Mk = it.M + (size_t)k * R * R;
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
            cplx acc = {0.0, 0.0};
            for (int a = 0; a < a_n; ++a) acc = cadd(acc, cmul(lenv[k][a], Mk[a * b_n + b]));
            lenv[k + 1][b] = acc;
        }
        __syncthreads();
    }
    // right environments: renv[k] = M_{k+1} ... M_{d-1} 1
    if (threadIdx.x == 0) renv[d - 1][0] = {1.0, 0.0};
    __syncthreads();
    for (int k = d - 1; k >= 1; --k) {
        const int a_n = it.crow[k], b_n = it.ccol[k];
        const cplx *Mk = it.M + (size_t)k * R * R;
        for (int a = threadIdx.x; a < a_n; a += blockDim.x) {
            cplx acc = {0.0, 0.0};
            for (int b = 0; b < b_n; ++b) acc = cadd(acc, cmul(Mk[a * b_n + b], renv[k][b]));
            renv[k - 1][a] = acc;
        }
        __syncthreads();
    }
    for (int k = 0; k < d; ++k) {
        const int a_n = it.crow[k], b_n = it.ccol[k];
        const cplx *M1 = it.M1 + (size_t)k * R * R;
        const cplx *M2 = it.M2 + (size_t)k * R * R;
        // mu1[k], mu2[k][k]
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
            cplx a1 = {0.0, 0.0}, a2 = {0.0, 0.0};
            for (int a = 0; a < a_n; ++a) {
                a1 = cadd(a1, cmul(lenv[k][a], M1[a * b_n + b]));
                a2 = cadd(a2, cmul(lenv[k][a], M2[a * b_n + b]));
            }
            v[b] = cmul(a1, renv[k][b]);
            w[b] = cmul(a2, renv[k][b]);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            cplx s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
            for (int b = 0; b < b_n; ++b) { s1 = cadd(s1, v[b]); s2 = cadd(s2, w[b]); }
            o[k] = s1;
            o[d + k * d + k] = s2;
        }
        __syncthreads();
        // mu2[k][l], l > k: carry lenv[k] M1_k through M_{k+1..l-1}
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
            cplx a1 = {0.0, 0.0};
            for (int a = 0; a < a_n; ++a) a1 = cadd(a1, cmul(lenv[k][a], M1[a * b_n + b]));
            v[b] = a1;
        }
        __syncthreads();
        for (int l = k + 1; l < d; ++l) {
            const int la = it.crow[l], lb = it.ccol[l];
            const cplx *L1 = it.M1 + (size_t)l * R * R;
            const cplx *L0 = it.M + (size_t)l * R * R;
            for (int b = threadIdx.x; b < lb; b += blockDim.x) {
                cplx acc = {0.0, 0.0};
                for (int a = 0; a < la; ++a) acc = cadd(acc, cmul(v[a], L1[a * lb + b]));
                w[b] = cmul(acc, renv[l][b]);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                cplx s = {0.0, 0.0};
                for (int b = 0; b < lb; ++b) s = cadd(s, w[b]);
                o[d + k * d + l] = s;
                o[d + l * d + k] = s;
            }
            __syncthreads();
            for (int b = threadIdx.x; b < lb; b += blockDim.x) {
                cplx acc = {0.0, 0.0};
                for (int a = 0; a < la; ++a) acc = cadd(acc, cmul(v[a], L0[a * lb + b]));
                w[b] = acc;
            }
            __syncthreads();
            for (int b = threadIdx.x; b < lb; b += blockDim.x) v[b] = w[b];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ tensor-train values at points
__global__ __launch_bounds__(64) void k_tt_values(const Item *items, int item, long long npts, const int *idx, cplx *out)
{
    __shared__ cplx v[TTFP_MAX_RANK], w[TTFP_MAX_RANK];
    const long long p = blockIdx.x;
    if (p >= npts) return;
    const Item &it = items[item];
    const int d = it.d, N = it.N, R = it.R;
    if (threadIdx.x == 0) v[0] = {1.0, 0.0};
    __syncthreads();
    for (int k = 0; k < d; ++k) {
        const int a_n = it.crow[k], b_n = it.ccol[k], i = idx[p * d + k];
        const cplx *core = it.cores + (size_t)k * R * N * R;
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) {
            cplx acc = {0.0, 0.0};
            for (int a = 0; a < a_n; ++a) acc = cadd(acc, cmul(v[a], core[((size_t)a * N + i) * b_n + b]));
            w[b] = acc;
        }
        __syncthreads();
        for (int b = threadIdx.x; b < b_n; b += blockDim.x) v[b] = w[b];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = v[0];
}

// ------------------------------------------------------------------ sampled error (convergence measure)
// The tensor train of an item against the integrand at n_samp uniformly drawn grid points
// (Sec. IV.B measures the convergence of the cross by the relative 1-norm error on random
// points): err_abs = sum_s |TT(x_s) - A(x_s)|, err_ref = sum_s |A(x_s)|. Coordinate k of point s
// is rand_index(seed, 7, s, k, N). One workgroup per item carries the row vectors v_s of a chunk
// of points through the cores, v_s <- v_s G_k(:, i_k(s), :): the points are bucketed by their
// node i_k (counting sort in LDS), and each bucket is one small product against the core slice
// G_k(:, i, :) on the FP64 matrix cores, so a slice is read once per 16 points of its bucket
// instead of once per point. The row vectors live in the item's fiber buffers (idle once the
// sweep has ended). Each point's value does not depend on the order inside its bucket, and the
// sums are formed per thread over a fixed set of points and reduced in thread order, so the
// result does not depend on scheduling.
constexpr int ERR_THREADS = 512;
constexpr int ERR_CHUNK = 8192;                    // points per pass through the cores
__global__ __launch_bounds__(ERR_THREADS) void k_err_est(Item *items, const int *active)
{
    __shared__ int cnt[MAXN + 1];
    __shared__ int cur[MAXN];
    __shared__ int perm[ERR_CHUNK];
    __shared__ double part[ERR_THREADS / 64][2];
    const int item = blockIdx.x;
    if (!active[item]) return;
    Item &it = items[item];
    const int ns = it.n_samp;
    if (ns <= 0) return;
    const int d = it.d, N = it.N, R = it.R;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = ERR_THREADS / 64;
    const int li = lane & 15, lk = lane >> 4;
    // points per chunk: the row vectors (chunk x R complex, twice) fit the fiber buffers
    const long long cap = (long long)it.rows_max * (R + it.p) / R;
    const int SC = (int)min((long long)ERR_CHUNK, cap);
    double sa = 0.0, sf = 0.0;
    for (int s0 = 0; s0 < ns; s0 += SC) {
        const int nsc = min(SC, ns - s0);
        cplx *V = it.F, *Wv = it.Qb;
        {
            const int b_n = it.ccol[0];
            const cplx *core = it.cores;
            for (int e = tid; e < nsc * b_n; e += ERR_THREADS) {
                const int jj = e / b_n, b = e - jj * b_n;
                const int i0 = rand_index(it.seed, 7, (uint64_t)(s0 + jj), 0, N);
                V[(size_t)jj * R + b] = core[(size_t)i0 * b_n + b];      // r_0 = 1
            }
        }
        __syncthreads();
        for (int k = 1; k < d; ++k) {
            const int a_n = it.crow[k], b_n = it.ccol[k];
            const cplx *core = it.cores + (size_t)k * R * N * R;
            // bucket the chunk's points by node i_k
            for (int q = tid; q <= N; q += ERR_THREADS) cnt[q] = 0;
            __syncthreads();
            for (int jj = tid; jj < nsc; jj += ERR_THREADS)
                atomicAdd(&cnt[rand_index(it.seed, 7, (uint64_t)(s0 + jj), (uint64_t)k, N)], 1);
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int q = 0; q < N; ++q) {
                    const int c = cnt[q];
                    cnt[q] = acc;
                    cur[q] = acc;
                    acc += c;
                }
                cnt[N] = acc;
            }
            __syncthreads();
            for (int jj = tid; jj < nsc; jj += ERR_THREADS) {
                const int i = rand_index(it.seed, 7, (uint64_t)(s0 + jj), (uint64_t)k, N);
                perm[atomicAdd(&cur[i], 1)] = jj;
            }
            __syncthreads();
            // bucket i: W[rows] = V[rows] G_k(:, i, :), 16 points per panel, one wave per bucket
            const int ntile = (b_n + 15) / 16;
            for (int i = wave; i < N; i += nw) {
                const int off = cnt[i], c = cnt[i + 1] - off;
                for (int p0 = 0; p0 < c; p0 += 16) {
                    double4_t prr[4], pii[4], pss[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        prr[q] = double4_t{0.0, 0.0, 0.0, 0.0};
                        pii[q] = prr[q];
                        pss[q] = prr[q];
                    }
                    const int rj = p0 + li < c ? perm[off + p0 + li] : -1;
                    for (int k0 = 0; k0 < a_n; k0 += 4) {
                        const int kk = k0 + lk;
                        const cplx a = (rj >= 0 && kk < a_n) ? V[(size_t)rj * R + kk] : cplx{0.0, 0.0};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if (q >= ntile) break;
                            const int cb = 16 * q + li;
                            const cplx b = (kk < a_n && cb < b_n) ? core[((size_t)kk * N + i) * b_n + cb] : cplx{0.0, 0.0};
                            prr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, prr[q], 0, 0, 0);
                            pii[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, pii[q], 0, 0, 0);
                            pss[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, pss[q], 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rp = p0 + lk + 4 * v;
                        if (rp >= c) continue;
                        const int jj = perm[off + rp];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if (q >= ntile) break;
                            const int cb = 16 * q + li;
                            if (cb < b_n)
                                Wv[(size_t)jj * R + cb] = {prr[q][v] - pii[q][v], pss[q][v] - prr[q][v] - pii[q][v]};
                        }
                    }
                }
            }
            __syncthreads();
            cplx *tmp = V;
            V = Wv;
            Wv = tmp;
        }
        // v_s is now the tensor train's value at x_s (r_d = 1)
        for (int jj = tid; jj < nsc; jj += ERR_THREADS) {
            int idx[MAXD];
            for (int k = 0; k < d; ++k) idx[k] = rand_index(it.seed, 7, (uint64_t)(s0 + jj), (uint64_t)k, N);
            const cplx f = integrand(it, idx);
            const cplx tt = V[(size_t)jj * R];
            sa += hypot(tt.x - f.x, tt.y - f.y);
            sf += hypot(f.x, f.y);
        }
        __syncthreads();
    }
    // thread partials in thread order
    sa = wave_sum(sa);
    sf = wave_sum(sf);
    if (lane == 0) {
        part[wave][0] = sa;
        part[wave][1] = sf;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, f = 0.0;
        for (int w = 0; w < nw; ++w) {
            a += part[w][0];
            f += part[w][1];
        }
        it.err_abs = a;
        it.err_ref = f;
    }
}

}  // namespace ttfp
