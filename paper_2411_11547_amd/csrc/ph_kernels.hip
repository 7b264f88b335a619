// HIP kernels of libpairhmm for gfx950 (CDNA4, wave64).
//
// The Pair-HMM forward recurrences (arXiv 2411.11547, Section II-A, Eq. 1-4)
// are swept along anti-diagonals inside one wavefront, after the paper's
// wavefront design (Section III-B): a group of P lanes computes one
// read/haplotype pair; lane t owns the K consecutive read rows
// tK+1 .. tK+K and keeps their M, I and D values in registers; at step s it
// updates column j = s - t + 1 of its rows and hands the values of its last
// row to lane t+1 with a DPP lane shift (the paper uses warp shuffles).  The
// haplotype is streamed through the lanes: every lane reads its column's
// code from a per-group ring buffer in LDS.  Emissions come from a
// per-lane table E[code][row] in LDS (Section III-B's E array).
//
// The FP32 sweeps carry rescaled states, It(i,j) = I(i,j) / delta_i and
// Dh(i,j) = D(i,j) / zeta_i, with alpha_i folded into the row's emission
// table (lam_ij = alpha_i * lambda_ij), so that a sum-product cell costs one
// LDS value and five VALU operations (the max-product cell, every sum a
// maximum, eight):
//
//   X  = M(i-1,j-1) + cD_i Dh(i-1,j-1) ;  X = cI_i It(i-1,j-1) + X
//   M(i,j)  = lam_ij X
//   It(i,j) = M(i-1,j) + kE_i It(i-1,j)
//   Dh(i,j) = M(i,j-1) + eps_i Dh(i,j-1)
//
// with cI_i = beta_i delta_{i-1} / alpha_i, cD_i = beta_i zeta_{i-1} /
// alpha_i and kE_i = eps_i delta_{i-1} / delta_i.  It and Dh are column and
// row sums of M with decaying weights, so they stay within the range of M
// unless delta falls steeply from one row to the next.  A read row with
// alpha_i < 2^-20 or kE_i > 2^20 (Phred gap-open qualities of 3 or less, or a
// gap-open quality rising by more than 60 from one base to the next, or
// explicit parameters like them) sends its pair to the FP64 sweep, which
// keeps the plain states with D pre-multiplied by the next row's beta:
//
//   X  = beta_i I(i-1,j-1) + Dt(i-1,j-1) ;  X = alpha_i M(i-1,j-1) + X
//   M(i,j) = lam_ij X
//   I(i,j) = delta_i M(i-1,j) + eps_i I(i-1,j)
//   Dt(i,j) = (beta_{i+1} zeta_i) M(i,j-1) + eps_i Dt(i,j-1)
//
// Differences from the paper's kernel:
//  * Rows past the read end are "absorbing".  Plain states: row m+1 has
//    lam = 0, delta = eps = 1, so I(m+1,j) = M(m,j) + I(m,j), and later rows
//    pass I down unchanged (delta = 0, eps = 1); the last register of the
//    group's last lane holds the quantity Section II-A sums into L, whatever
//    m is.  Rescaled states: row m+1 has lam = 1, cD = 0 and cI = delta_m,
//    so M(m+1,j) = M(m,j-1) + I(m,j-1), and its Dh (eps = 1) sums that along
//    the row (max-product: keeps its running maximum): the row-(m+1) lane
//    flushes it into an FP64 accumulator every chunk of the haplotype ring
//    (32 or 64 steps).  Later rows have every coefficient 0: their M and Dh
//    are exactly zero, and so is It from row m+3 on.  (The paper pads reads
//    with N, which would change L if read at row pK.)
//  * Columns past the haplotype end carry a PAD code whose emission is 0, so
//    groups of one wave may have different n and still add only exact zeros.
//  * D(0, j) = 1/n is scaled by 2^120 (FP32) or 2^1020 (FP64) so that the
//    sweep stays inside the normal range; pairs whose scaled FP32 sum falls
//    below a threshold are queued and recomputed by the FP64 sweep.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ph_internal.h"
#include "ph_device.h"

namespace ph {

__constant__ double c_prob[256];  // Phred q -> 10^(-q/10), computed on the host in FP64
// the same table rounded to FP32, and 1 - p, p / 3 formed in FP64 then rounded
__constant__ float c_pf[256], c_1mpf[256], c_pd3f[256];

hipError_t upload_luts()
{
    double t[256];
    float f[256], g[256], h[256];
    for (int q = 0; q < 256; ++q) {
        t[q] = pow(10.0, -(double)q / 10.0);
        f[q] = (float)t[q];
        g[q] = (float)(1.0 - t[q]);
        h[q] = (float)(t[q] / 3.0);
    }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_prob), t, sizeof(t));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pf), f, sizeof(f));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_1mpf), g, sizeof(g));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pd3f), h, sizeof(h));
    return e;
}

// Per-lane LDS layout for one configuration: E[code][plane][lane] of 8-byte
// entries (two FP32 rows or one FP64 row per plane), then the haplotype
// rings of the groups.  Entry (c, q, lane) sits at
// c*CODE_BYTES + q*512 + lane*8, so 64 lanes read 512 consecutive bytes when
// they look up the same code and never conflict when they look up different
// codes.
template <typename T, int P, int K>
struct Cfg {
    static constexpr int G = 64 / P;
    static constexpr int RPP = 8 / (int)sizeof(T);  // rows per plane entry
    static constexpr int NPL = (K + RPP - 1) / RPP;
    static constexpr int KP = NPL * RPP;
    static constexpr int CODE_BYTES = NPL * 512;
    static constexpr int E_BYTES = kCodes * CODE_BYTES;
    static constexpr int RING_BYTES = ring_alloc(P) * 2;  // u16 E-table offsets
    static constexpr int LDS_BYTES = E_BYTES + G * RING_BYTES;
};

template <typename T, int P, int K>
__device__ __forceinline__ void load_lam(T *lam, const char *ebase)
{
    using C = Cfg<T, P, K>;
#pragma unroll
    for (int q = 0; q < C::NPL; ++q) {
        if constexpr (sizeof(T) == 4) {
            float2 v = *(const float2 *)(ebase + q * 512);
            lam[2 * q] = v.x;
            lam[2 * q + 1] = v.y;
        } else {
            lam[q] = *(const double *)(ebase + q * 512);
        }
    }
}

// Chunk `chunk` (ring_chunk(P) columns) of the group's haplotype goes into its ring
// as byte offsets of the code's E table (code * code_bytes), in two parts so
// that the global-load latency overlaps a chunk of the sweep: ring_load
// issues lane t's loads into registers (0xffff marks a column past the
// haplotype end; nothing waits on the loads here), ring_store converts and
// writes them.  Chunk c + 2 is loaded at the start of the sweep's chunk c and
// written at its end, into the slot of chunk c - 2, which no lane reads after
// the sweep's chunk c (lane 63 of a 64-lane group, the furthest behind,
// reads chunk c - 1 during chunk c).  Each lane takes ring_chunk(P) / P
// columns.
template <int P>
struct RingPer {
    static constexpr int CH = ring_chunk(P);
    static constexpr int N = CH / P;
    static_assert(N >= 1, "a chunk has at least one column per lane");
};

template <int P>
__device__ __forceinline__ void ring_load(uint32_t (&c)[RingPer<P>::N], int chunk, const uint8_t *hap, int n, int t)
{
    constexpr int PER = RingPer<P>::N;
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int col = chunk * RingPer<P>::CH + t * PER + b;
        c[b] = col < n ? (uint32_t)hap[col] : 0xffffu;
    }
}

// (a chain's code stream holds codes 0..5 already: PAD stays PAD)
template <int P>
__device__ __forceinline__ void ring_store(uint16_t *ring, int chunk, const uint32_t (&c)[RingPer<P>::N], int t,
                                           int code_bytes, bool coded = false)
{
    constexpr int PER = RingPer<P>::N, CH = RingPer<P>::CH;
    const int slot = chunk & 3;
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int x = t * PER + b;
        const uint32_t code = c[b] == 0xffffu ? (uint32_t)kPad : coded ? c[b] : clamp_code(c[b]);
        const uint16_t off = (uint16_t)(code * code_bytes);
        ring[slot * CH + x] = off;
        if (slot == 0) ring[4 * CH + x] = off;
    }
}

enum { kModeBinned = 0, kModePlain = 1, kModeRescue = 2 };

// One anti-diagonal step of a lane: column j = s - t + 1 of rows tK+1..tK+K.
// M, I, D hold column j-1 on entry and column j on exit; (Md, Id, Dd) are the
// values of the row above the lane's first row at column j-1, received from
// lane t-1 at the previous step.  The D shift folds into one v_add_f32_dpp
// with the row-0 edge value.
//
// Windowed mode (W): the first lane's row above is a stored boundary row;
// (tM, tI, edge) are its M, I and D at column j, zero in the other lanes.
//
// Viterbi mode (V): the max-product form of Eq. (1)-(3), every sum over
// predecessor states a maximum (beta >= 0, so the pre-multiplied D still
// folds in: beta max(I, D) = max(beta I, beta D)); the row-m accumulator
// keeps the maximum instead of the sum.
//
// epI0 is the first row's eps in its I term (the one that multiplies the
// value received from above); it differs from ep[0] only in the first lane
// of a group, where it is 0 (see the prologue).
template <typename T, int P, int K, bool W = false, bool V = false>
__device__ __forceinline__ void cell_step(T (&M)[K], T (&I)[K], T (&D)[K], T &Md, T &Id, T &Dd, const T *lam,
                                          const T (&al)[K], const T (&be)[K], const T (&de)[K],
                                          const T (&ep)[K], const T (&zt)[K], T epI0, T edge, T &acc,
                                          T tM = 0, T tI = 0)
{
    T Mu = shift_up<P>(M[K - 1]);
    T Iu = shift_up<P>(I[K - 1]);
    const T Du = shift_up<P>(D[K - 1]) + edge;
    if constexpr (W) {
        Mu += tM;
        Iu += tI;
    }
    T mup = Mu, iup = Iu, mdg = Md, idg = Id, ddg = Dd;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const T mo = M[r], io = I[r], dol = D[r];
        T mn, in, dn;
        const T epi = r == 0 ? epI0 : ep[r];
        if constexpr (V) {
            mn = lam[r] * fmax(fmax(al[r] * mdg, be[r] * idg), ddg);
            in = fmax(de[r] * mup, epi * iup);
            dn = fmax(zt[r] * mo, ep[r] * dol);
        } else {
            T x = fma(be[r], idg, ddg);
            x = fma(al[r], mdg, x);
            mn = lam[r] * x;
            in = fma(epi, iup, de[r] * mup);
            dn = fma(ep[r], dol, zt[r] * mo);
        }
        M[r] = mn;
        I[r] = in;
        D[r] = dn;
        mdg = mo;
        idg = io;
        ddg = dol;
        mup = mn;
        iup = in;
    }
    Md = Mu;
    Id = Iu;
    Dd = Du;
    if constexpr (V)
        acc = fmax(acc, I[K - 1]);
    else
        acc += I[K - 1];
}

// Maximum of two non-negative floats (every max-product state and
// coefficient of the rescaled sweep is >= 0): their bit patterns order like
// unsigned integers, so the integer maximum needs none of the canonicalising
// moves a float maximum gets for operands the compiler cannot prove canonical.
__device__ __forceinline__ float max_nonneg(float a, float b)
{
    return __builtin_bit_cast(float, max(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)));
}

// The same step with the rescaled states (M, It, Dh) of the FP32 sweeps;
// lam holds alpha_i lambda_ij, ci, cd, ke and ep the coefficients cI, cD, kE
// and eps of the file header.  (eM, eI, eD) are added to the values received
// from the lane above: the first lane's row-0 boundary (eI = beta_1 / n,
// scaled, enters through It with cI = 1 on the read's first row) or, in
// windowed mode, the stored boundary row; zero in the other lanes.
//
// Groups of 4 and 8 lanes: the first lane of a group other than lanes 0, 16,
// 32, 48 receives the previous group's last row, which may be that pair's
// absorbing row or the row below it.  keep is 0 in the first lane of every
// group and all ones elsewhere; it clears the received M and It there.  The
// received Dh needs no mask: it meets cD = 0 on the read's first row.
//
// Viterbi mode (V): every sum a maximum, as in cell_step; the rescaling by
// positive per-row factors commutes with the maximum, and every value is
// non-negative (max_nonneg).
template <typename T, int P, int K, bool W = false, bool V = false>
__device__ __forceinline__ void cell_step_hat(T (&M)[K], T (&I)[K], T (&D)[K], T &Md, T &Id, T &Dd,
                                              const T *lam, const T (&ci)[K], const T (&cd)[K],
                                              const T (&ke)[K], const T (&ep)[K], T eI, uint32_t keep,
                                              T eM = 0, T eD = 0)
{
    T Mu = shift_up<P>(M[K - 1]);
    T Iu = shift_up<P>(I[K - 1]);
    T Du = shift_up<P>(D[K - 1]);
    if constexpr (P < 16) {
        Mu = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, Mu) & keep);
        Iu = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, Iu) & keep);
    }
    Iu += eI;
    if constexpr (W) {
        Mu += eM;
        Du += eD;
    }
    T mup = Mu, iup = Iu, mdg = Md, idg = Id, ddg = Dd;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const T mo = M[r], io = I[r], dol = D[r];
        T mn, in, dn;
        if constexpr (V) {
            mn = lam[r] * max_nonneg(max_nonneg(mdg, ci[r] * idg), cd[r] * ddg);
            in = max_nonneg(mup, ke[r] * iup);
            dn = max_nonneg(mo, ep[r] * dol);
        } else {
            T x = fma(cd[r], ddg, mdg);
            x = fma(ci[r], idg, x);
            mn = lam[r] * x;
            in = fma(ke[r], iup, mup);
            dn = fma(ep[r], dol, mo);
        }
        M[r] = mn;
        I[r] = in;
        D[r] = dn;
        mdg = mo;
        idg = io;
        ddg = dol;
        mup = mn;
        iup = in;
    }
    Md = Mu;
    Id = Iu;
    Dd = Du;
}

// cell_step_hat with the first row's sums formed by the lane above: at the
// start of a step every lane forms, from its last row's (M, It, Dh) at its
// column, the two sums the next lane's first row needs,
//   X = M + cD' Dh + cI' It  and  Y = M + kE' It
// with the next lane's first-row coefficients (cib, cdb, keb), and hands on
// X and Y instead of the three states: two lane shifts per step instead of
// three (four DPP moves instead of six in FP64).  The receiving row then
// costs M = lam X (X of the step before, held in Xd), It = Y and the Dh
// update; the sums are the same operations in the same order as in
// cell_step_hat, so the results are bit-identical.  In the first lane of a
// group X is the row-0 boundary value eX (the It edge, cI = 1 on the read's
// first row; Xd starts at eX) and Y is 0 (kE = 0 there).  Not used by the
// windowed sweep, whose first lane takes a stored row.
template <typename T, int P, int K, bool V = false>
__device__ __forceinline__ void cell_step_hx(T (&M)[K], T (&I)[K], T (&D)[K], T &Xd, const T *lam,
                                             const T (&ci)[K], const T (&cd)[K], const T (&ke)[K],
                                             const T (&ep)[K], T cib, T cdb, T keb, T eX, uint32_t keep)
{
    T X, Y;
    if constexpr (V) {
        X = max_nonneg(max_nonneg(M[K - 1], cib * I[K - 1]), cdb * D[K - 1]);
        Y = max_nonneg(M[K - 1], keb * I[K - 1]);
    } else {
        X = fma(cib, I[K - 1], fma(cdb, D[K - 1], M[K - 1]));
        Y = fma(keb, I[K - 1], M[K - 1]);
    }
    T Yu = shift_up<P>(Y);
    if constexpr (P < 16) Yu = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, Yu) & keep);
    T mdg = M[0], idg = I[0], ddg = D[0];
    M[0] = lam[0] * Xd;
    if constexpr (P < 16) {
        Xd = __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, shift_up<P>(X)) & keep) + eX;
    } else {
        // the first lane keeps its X, which is eX at every step
        Xd = shift_up_or<P>(Xd, X);
    }
    I[0] = Yu;
    if constexpr (V)
        D[0] = max_nonneg(mdg, ep[0] * ddg);
    else
        D[0] = fma(ep[0], ddg, mdg);
    T mup = M[0], iup = I[0];
#pragma unroll
    for (int r = 1; r < K; ++r) {
        const T mo = M[r], io = I[r], dol = D[r];
        T mn, in, dn;
        if constexpr (V) {
            mn = lam[r] * max_nonneg(max_nonneg(mdg, ci[r] * idg), cd[r] * ddg);
            in = max_nonneg(mup, ke[r] * iup);
            dn = max_nonneg(mo, ep[r] * dol);
        } else {
            T x = fma(cd[r], ddg, mdg);
            x = fma(ci[r], idg, x);
            mn = lam[r] * x;
            in = fma(ke[r], iup, mup);
            dn = fma(ep[r], dol, mo);
        }
        M[r] = mn;
        I[r] = in;
        D[r] = dn;
        mdg = mo;
        idg = io;
        ddg = dol;
        mup = mn;
        iup = in;
    }
}

// lane t receives lane t+1's value over the whole wave (lane 63: 0)
__device__ __forceinline__ float from_next_lane(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130 /* wave_shl:1 */,
                                                              0xf, 0xf, true));
}
__device__ __forceinline__ double from_next_lane(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x130, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One step of the windowed sweep (64 lanes): lane 0 takes the staged
// boundary values of its column, and the last lane writes the window's last
// row at its column back to the boundary slot unless this is the final window.
template <typename T, int K, bool V>
__device__ __forceinline__ void window_step(T (&M)[K], T (&I)[K], T (&D)[K], T &Md, T &Id, T &Dd, const T *lam,
                                            const T (&al)[K], const T (&be)[K], const T (&de)[K],
                                            const T (&ep)[K], const T (&zt)[K], T epI0, T edge, T &acc,
                                            const T *top, int u, int t, bool fin, T *bnd, int s, int n)
{
    const T tM = top[u], tI = top[64 + u], tD = top[128 + u];
    const bool first = t == 0;
    cell_step<T, 64, K, true, V>(M, I, D, Md, Id, Dd, lam, al, be, de, ep, zt, epI0, first ? tD + edge : (T)0,
                                 acc, first ? tM : (T)0, first ? tI : (T)0);
    const int j = s - 62;  // the last lane's column
    if (!fin && t == 63 && j >= 1 && j <= n) {
        T *b = bnd + (int64_t)j * 3;
        b[0] = M[K - 1];
        b[1] = I[K - 1];
        b[2] = D[K - 1];
    }
}

// window_step with the rescaled states: the staged boundary row holds
// (M, It, Dh) and the row-0 boundary enters through It.
template <typename T, int K, bool V>
__device__ __forceinline__ void window_step_hat(T (&M)[K], T (&I)[K], T (&D)[K], T &Md, T &Id, T &Dd,
                                                const T *lam, const T (&ci)[K], const T (&cd)[K],
                                                const T (&ke)[K], const T (&ep)[K], T edge, const T *top, int u,
                                                int t, bool fin, T *bnd, int s, int n)
{
    const T tM = top[u], tI = top[64 + u], tD = top[128 + u];
    const bool first = t == 0;
    cell_step_hat<T, 64, K, true, V>(M, I, D, Md, Id, Dd, lam, ci, cd, ke, ep, first ? tI + edge : (T)0, ~0u,
                                     first ? tM : (T)0, first ? tD : (T)0);
    const int j = s - 62;  // the last lane's column
    if (!fin && t == 63 && j >= 1 && j <= n) {
        T *b = bnd + (int64_t)j * 3;
        b[0] = M[K - 1];
        b[1] = I[K - 1];
        b[2] = D[K - 1];
    }
}

// Coefficients of the rescaled states for read row i >= 1 (0-based) from
// its delta, zeta, eps, beta and the row above's delta and zeta: the factor
// alpha_i that goes into the row's emissions, cI, cD and kE.  Returns false
// when the row is outside what the FP32 states carry (alpha_i < 2^-20 or
// kE > 2^20); the coefficients are then 0 and the pair goes to the FP64
// sweep.  FP32 form for Phred qualities (alpha = 1 - delta - zeta rounded in
// FP32), FP64 form for explicit parameters; the sweep's prologue and the
// windowed sweep's check of earlier windows call the same functions.
__device__ __forceinline__ bool hat_coef(float dp, float zp, float d, float z, float e, float b, float &fac,
                                         float &ci, float &cd, float &ke)
{
    const float a = 1.0f - d - z;
    const float ra = __builtin_amdgcn_rcpf(a);
    const float k = e * dp * __builtin_amdgcn_rcpf(d);
    const bool ok = a >= 0x1p-20f && k <= 0x1p20f;
    fac = a;
    ci = ok ? b * dp * ra : 0.0f;
    cd = ok ? b * zp * ra : 0.0f;
    ke = ok ? k : 0.0f;
    return ok;
}

__device__ __forceinline__ bool hat_coef(const RowPar &p, const RowPar &pp, double &fac, double &ci, double &cd,
                                         double &ke)
{
    const double k = p.e * pp.d / p.d;
    const bool ok = p.a >= 0x1p-20 && k <= 0x1p20;
    fac = p.a;
    ci = ok ? p.b * pp.d / p.a : 0.0;
    cd = ok ? p.b * pp.z / p.a : 0.0;
    ke = ok ? k : 0.0;
    return ok;
}

// read row i >= 1 (0-based) at read offset ro cannot be carried by the FP32
// rescaled states (see hat_coef)
__device__ __forceinline__ bool hat_row_unsafe(const DevProblem &pb, const double *lin, int64_t ro, int i)
{
    if (lin) {
        double fac, ci, cd, ke;
        return !hat_coef(load_row(pb, lin, ro + i, c_prob), load_row(pb, lin, ro + i - 1, c_prob), fac, ci, cd,
                         ke);
    }
    float fac, ci, cd, ke;
    const int64_t pos = ro + i;
    return !hat_coef(c_pf[pb.iq[pos - 1]], c_pf[pb.dq[pos - 1]], c_pf[pb.iq[pos]], c_pf[pb.dq[pos]],
                     c_pf[pb.gq[pos]], c_1mpf[pb.gq[pos]], fac, ci, cd, ke);
}

// Start scale of the rescaled states: FP32 2^120 (as the plain states); FP64
// 2^1000, lower than the plain FP64 sweep's 2^1020 so that It and Dh, which
// can exceed the largest M by a few binary orders, stay finite.
template <typename T>
struct RangeHat;
template <>
struct RangeHat<float> {
    static constexpr int kExp = 120;
};
template <>
struct RangeHat<double> {
    static constexpr int kExp = 1000;
};

// Sweep one tile: up to G = 64/P pairs, one per lane group.  Group g takes
// record rec_first + g (or rec_idx_list[rec_first + g]) if g < nvalid.
//
// H: rescaled states (M, It, Dh).  The FP32 sweeps always use them; the
// FP64 sweep uses them for pairs that left the FP32 range (FP64 rescaled
// sweep) and the plain states for pairs with a row outside the rescaled
// states and for what the rescaled FP64 sweep passes on (plain FP64 sweep).
//
// Windowed mode (W, reads longer than kMaxReadLen; P = 64, one pair per
// wave): the launch covers rows A.window * kLongRows + 1 .. + kLongRows of
// the pair.  Its top boundary row (the states of the row above, columns
// 0..n) is read from the pair's slot `bnd_slot` of A.bnd, staged a chunk
// at a time in LDS, and the window's last row is written back in place
// (column j is read at step j-1 and written at step j+62).  Only the window
// that holds the absorbing row m+1 produces the result.
template <typename T, int P, int K, bool W = false, bool V = false, bool H = sizeof(T) == 4>
__device__ void sweep_tile(const SweepArgs &A, const int32_t *rec_idx_list, int rec_first,
                           int nvalid, char *lds, int bnd_slot = 0)
{
    using C = Cfg<T, P, K>;
    static_assert(!W || (P == 64 && K * P == kLongRows), "windowed sweep: 64 lanes x kLongRows / 64 rows");
    static_assert(sizeof(T) == 4 || !H || (!W && !V), "FP64 rescaled states: the binned sum-product sweep only");
    constexpr bool HAT = H;  // rescaled states (M, It, Dh)
    constexpr int kExp = HAT ? RangeHat<T>::kExp : Range<T>::kExp;
    const int lane = threadIdx.x;
    const int g = lane / P;
    const int t = lane % P;
    const int r0 = W ? A.window * kLongRows : 0;  // first row of the window (0-based)
    bool gvalid = g < nvalid;
    const int ridx = gvalid ? (rec_idx_list ? rec_idx_list[rec_first + g] : rec_first + g) : 0;

    PairRec rec = {0, 0, 0, 0};
    if (gvalid) rec = A.recs[ridx];
    const DevProblem &pb = A.pb;
    const double *lin = A.lin_params;
    const int64_t ro = gvalid ? pb.read_offset[rec.read] : 0;
    const int m = gvalid ? (int)(pb.read_offset[rec.read + 1] - ro) : 0;
    if constexpr (W) {
        // a pair whose absorbing row lies in an earlier window is done
        gvalid = gvalid && m >= r0;
        if (!__builtin_amdgcn_readfirstlane((int)gvalid)) return;
    }
    const bool fin = !W || m < r0 + kLongRows;  // this window holds row m + 1
    // Chain tile (FP32 binned sweep, records with n < 0): every group of the
    // tile sweeps its read against the same NH haplotypes h0, h0 + 1, ... of
    // its batch in turn, along their code stream; lane i holds the length of
    // haplotype h0 + i, Lc is the stream's length up to the last haplotype's end.
    constexpr bool CHN = kChains && HAT && !W && sizeof(T) == 4;
    bool chain = false;
    int NH = 1, h0 = 0, nvec = 0, Lc = 0;
    if constexpr (CHN) {
        const int r0n = __builtin_amdgcn_readfirstlane(rec.n);
        chain = r0n < 0;
        if (chain) {
            NH = -r0n;
            h0 = __builtin_amdgcn_readfirstlane(rec.hap);
            if (lane < NH) nvec = (int)(pb.hap_offset[h0 + lane + 1] - pb.hap_offset[h0 + lane]);
            int sum = nvec;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) sum += __shfl_xor(sum, off);
            Lc = __builtin_amdgcn_readfirstlane(sum) + kChainSep * (NH - 1);
        }
    }
    const int n = chain ? __builtin_amdgcn_readlane(nvec, 0) : gvalid ? rec.n : 0;
    const int64_t ho = gvalid ? pb.hap_offset[rec.hap] : 0;
    const uint8_t *hap = chain ? A.chain_codes + ho + (int64_t)kChainSep * h0 : pb.hap_bases + ho;
    const int nring = chain ? Lc : n;  // columns of the ring's source
    T *bnd = W ? (T *)A.bnd + (int64_t)bnd_slot * A.bnd_stride : nullptr;
    T *top = (T *)(lds + C::E_BYTES + C::G * C::RING_BYTES);  // windowed: [3][64] staged boundary values

    // the longest haplotype (chain) of the wave sets the number of steps
    int nmax = nring;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) nmax = max(nmax, __shfl_xor(nmax, off));
    nmax = __builtin_amdgcn_readfirstlane(nmax);

    // ---- prologue: parameters of my rows, my slice of the E table ----------
    // Loads use clamped row indices so that they stay inside the read;
    // padding rows then get their absorbing parameters by select.  With the
    // rescaled states the read's first row has cI = 1 and cD = kE = 0 (the
    // row above it is the DP boundary: M = I = 0, its D enters as the It edge
    // value), the absorbing row m (0-based) has lam = 1 for every code,
    // cI = delta_{m-1}, cD = kE = 0 and eps = 1, and the rows past it have
    // every coefficient 0.
    char *E = lds;
    char *mine = E + lane * 8;
    uint16_t *ring = (uint16_t *)(lds + C::E_BYTES + g * C::RING_BYTES);
    auto slot = [&](int c, int r) -> T * {
        return (T *)(mine + c * C::CODE_BYTES + (r / C::RPP) * 512 + (r % C::RPP) * (int)sizeof(T));
    };
    const int mload = m > 0 ? m : 1;
    const int base = r0 + t * K;  // my first row (0-based)
    T al[K], be[K], de[K], ep[K], zt[K];  // plain states
    T ci[K], cd[K], ke[K];                // rescaled states (with ep)
    T edge = 0;
    float e0f = 0.0f;   // FP32: the edge value times n (chains: divided by each haplotype's n)
    bool bad = false;  // rescaled states: one of my rows is outside what they carry
    bool phred32 = false;  // the FP32 sweep in Phred mode (rescaled states)
    if constexpr (HAT && sizeof(T) == 4) phred32 = lin == nullptr;
    if (phred32) {
      if constexpr (HAT && sizeof(T) == 4) {
        // FP32 sweep, Phred mode: all of the lane's loads issued at once,
        // decoded through the FP32 tables (1 - p and p/3 rounded from FP64);
        // the transition parameters first, then the E table with each real
        // row's alpha folded in
        uint32_t bq[C::KP], code[C::KP], iq[K + 1], dq[K + 1], gq[K];
#pragma unroll
        for (int r = 0; r < C::KP; ++r) {
            const int64_t pos = ro + min(base + r, mload - 1);
            bq[r] = pb.bq[pos];
            code[r] = clamp_code(pb.read_bases[pos]);
        }
        // iq[r], dq[r]: row base + r - 1 (the row above row r); gq[r]: row base + r
#pragma unroll
        for (int r = 0; r <= K; ++r) {
            const int64_t pa = ro + min(max(base + r - 1, 0), mload - 1);
            iq[r] = pb.iq[pa];
            dq[r] = pb.dq[pa];
            if (r < K) gq[r] = pb.gq[ro + min(base + r, mload - 1)];
        }
        float fac[C::KP];
#pragma unroll
        for (int r = 0; r < C::KP; ++r) fac[r] = 0.0f;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int i = base + r;
            const bool real = i < m;
            const float e = c_pf[gq[r]];
            float f, c1, c2, k;
            const bool ok = hat_coef(c_pf[iq[r]], c_pf[dq[r]], c_pf[iq[r + 1]], c_pf[dq[r + 1]], e,
                                     c_1mpf[gq[r]], f, c1, c2, k);
            const bool inner = real && i >= 1;
            bad = bad || (inner && !ok);
            // a row outside the FP32 states gets zero emissions: its pair is
            // recomputed in FP64, and every FP32 value stays >= 0 (alpha may
            // be negative there), which the max-product sweep relies on
            fac[r] = inner ? (ok ? f : 0.0f) : 1.0f;
            ci[r] = inner ? c1 : i == 0 ? 1.0f : i == m ? c_pf[iq[r]] : 0.0f;
            cd[r] = inner ? c2 : 0.0f;
            ke[r] = inner ? k : 0.0f;
            ep[r] = real ? e : (i == m ? 1.0f : 0.0f);
        }
        if (t == 0 && m > 0 && r0 == 0) {
            e0f = ldexpf(c_1mpf[gq[0]], kExp);
            edge = e0f / (float)n;
        }
#pragma unroll
        for (int q = 0; q < C::NPL; ++q) {
            float lm[C::RPP], lx[C::RPP];
            bool one[C::RPP];
#pragma unroll
            for (int rr = 0; rr < C::RPP; ++rr) {
                const int r = q * C::RPP + rr;
                const bool real = (r < K) && (base + r < m);
                one[rr] = HAT && (r < K) && (base + r == m);
                lm[rr] = real ? c_1mpf[bq[r]] * fac[r] : 0.f;
                lx[rr] = real ? c_pd3f[bq[r]] * fac[r] : 0.f;
            }
#pragma unroll
            for (int c = 0; c < kCodes; ++c) {
                T v[C::RPP];
#pragma unroll
                for (int rr = 0; rr < C::RPP; ++rr) {
                    const int r = q * C::RPP + rr;
                    const bool match = code[r] == (uint32_t)c || code[r] == 4u || c == 4;
                    v[rr] = one[rr] ? (T)1 : c == kPad ? (T)0 : (T)(match ? lm[rr] : lx[rr]);
                }
                if constexpr (sizeof(T) == 4)
                    *(float2 *)(mine + c * C::CODE_BYTES + q * 512) = make_float2(v[0], v[1]);
                else
                    *(double *)(mine + c * C::CODE_BYTES + q * 512) = v[0];
            }
        }
      }
    } else {
        // FP64 sweep or explicit parameters: one row at a time in FP64, the
        // row parameters parked in the lane's own E entries, then loaded
#pragma unroll 1
        for (int r = 0; r < K; ++r) {
            const int i = base + r;
            const int ic = min(i, mload - 1);
            const RowPar p = load_row(pb, lin, ro + ic, c_prob);
            const bool real = i < m;
            if constexpr (HAT) {
                const bool inner = real && i >= 1;
                const RowPar pp = load_row(pb, lin, ro + min(max(i - 1, 0), mload - 1), c_prob);
                double f, c1, c2, k;
                const bool ok = hat_coef(p, pp, f, c1, c2, k);
                bad = bad || (inner && !ok);
                *slot(0, r) = inner ? (T)c1 : i == 0 ? (T)1 : i == m ? (T)pp.d : (T)0;
                *slot(1, r) = inner ? (T)c2 : (T)0;
                *slot(2, r) = inner ? (T)k : (T)0;
                *slot(3, r) = real ? (T)p.e : (i == m ? (T)1 : (T)0);
                // alpha folded into the row's emissions, zero on a row outside
                // the FP32 states (as in the Phred branch)
                *slot(4, r) = inner ? (ok ? (T)f : (T)0) : (T)1;
            } else {
                const double bn = load_beta(pb, lin, ro + min(i + 1, mload - 1), c_prob);
                *slot(0, r) = real ? (T)p.a : (T)0;
                *slot(1, r) = real ? (T)p.b : (T)0;
                *slot(2, r) = real ? (T)p.d : (i == m ? (T)1 : (T)0);
                *slot(3, r) = real ? (T)p.e : (T)1;
                *slot(4, r) = (real && i + 1 < m) ? (T)(bn * p.z) : (T)0;
            }
        }
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if constexpr (HAT) {
                ci[r] = *slot(0, r);
                cd[r] = *slot(1, r);
                ke[r] = *slot(2, r);
                ep[r] = *slot(3, r);
            } else {
                al[r] = *slot(0, r);
                be[r] = *slot(1, r);
                de[r] = *slot(2, r);
                ep[r] = *slot(3, r);
                zt[r] = *slot(4, r);
            }
        }
        if (t == 0 && m > 0 && r0 == 0) {
            if constexpr (sizeof(T) == 4) {
                e0f = (float)ldexp(load_beta(pb, lin, ro, c_prob), kExp);
                edge = e0f / (float)n;
            } else {
                edge = (T)(ldexp(load_beta(pb, lin, ro, c_prob), kExp) / (double)n);
            }
        }
        // E[c][row] = lam of the row against haplotype code c (N matches all,
        // PAD = 0); rescaled states: times alpha on the read's rows after the first
#pragma unroll 1
        for (int r = 0; r < C::KP; ++r) {
            const int i = base + r;
            const int ic = min(i, mload - 1);
            const RowPar p = load_row(pb, lin, ro + ic, c_prob);
            const bool real = (r < K) && (i < m);
            const bool one = HAT && (r < K) && (i == m);
            // read before this row's entries are written
            const double f = (HAT && real) ? (double)*slot(4, r) : 1.0;
            const uint32_t code = clamp_code(pb.read_bases[ro + ic]);
            const T lm = real ? (T)(p.lm * f) : (T)0, lx = real ? (T)(p.lx * f) : (T)0;
#pragma unroll
            for (int c = 0; c < kCodes; ++c) {
                const bool match = code == (uint32_t)c || code == 4u || c == 4;
                *slot(c, r) = one ? (T)1 : c == kPad ? (T)0 : (match ? lm : lx);
            }
        }
    }
    // Plain states: the first lane of a group takes the row above its first
    // row from the boundary of the DP (row 0: M = I = 0, D = 1/n), but in
    // groups of 4 or 8 lanes the lane shift hands it the previous group's last
    // row instead.  That row is an absorbing row (rows past m: M = 0 and D = 0
    // exactly), so its M and D terms vanish by themselves; its I enters the
    // first row only through beta (with the diagonal) and eps (from above),
    // and both are set to 0 here, which is exact because row 0 has I = 0.  In
    // later windows of a long read the row above is a real stored row and
    // keeps its terms.  (Rescaled states: the received M and It are cleared
    // in the first lane of each group, see cell_step_hat.)
    T epI0 = ep[0];
    if constexpr (!HAT) {
        if (t == 0 && r0 == 0) {
            be[0] = 0;
            epI0 = 0;
        }
    }
    const uint32_t keep = t == 0 ? 0u : ~0u;
    // rescaled states: the pair goes to the FP64 sweep if any of its rows is
    // outside what they carry (rows of earlier windows are checked by the
    // final one)
    bool gbad = false;
    if constexpr (HAT) {
        if constexpr (W) {
            if (fin)
                for (int i = 1 + t; i < r0; i += 64) bad = bad || hat_row_unsafe(pb, lin, ro, i);
        }
        const uint64_t bm = __ballot(bad);
        const uint64_t gm = P == 64 ? ~0ull : (((1ull << P) - 1) << (g * P));
        gbad = (bm & gm) != 0;
    }
    // haplotype ring: PAD everywhere (negative columns read slot 3), then chunks 0 and 1
    for (int x = t; x < ring_alloc(P); x += P) ring[x] = (uint16_t)(kPad * C::CODE_BYTES);
    __syncthreads();
    {
        uint32_t c0[RingPer<P>::N], c1[RingPer<P>::N];
        ring_load<P>(c0, 0, hap, nring, t);
        ring_load<P>(c1, 1, hap, nring, t);
        ring_store<P>(ring, 0, c0, t, C::CODE_BYTES, chain);
        ring_store<P>(ring, 1, c1, t, C::CODE_BYTES, chain);
    }
    __syncthreads();

    // ---- sweep ----------------------------------------------------------------
    T M[K], I[K], D[K];
#pragma unroll
    for (int r = 0; r < K; ++r) M[r] = I[r] = D[r] = 0;
    // row above the lane's first row at column j-1 = 0: the first lane's
    // row-0 boundary (the edge value) sits in It (rescaled) or Dt (plain)
    T Md = 0, Id = HAT ? edge : (T)0, Dd = HAT ? (T)0 : edge;
    // rescaled states outside the windowed sweep (cell_step_hx): the first
    // row's X at column 0, and the next lane's first-row coefficients
    T Xd = edge, cib = 0, cdb = 0, keb = 0;
    if constexpr (HAT && !W) {
        cib = from_next_lane(ci[0]);
        cdb = from_next_lane(cd[0]);
        keb = from_next_lane(ke[0]);
    }
    // row-m sum (Viterbi: maximum).  Plain states: each chunk of CH steps
    // in T, then FP64.  Rescaled states: the absorbing row's Dh, flushed
    // into FP64 every CH steps by the lane that holds it (row index rml).
    constexpr int CH = ring_chunk(P);
    double acc = 0.0;
    const int rml = m - base;
    // steps run in pairs; a step past the last column only meets PAD columns
    // in the last lane and adds exact zeros.  The last lane reaches column
    // nmax after nmax + P - 1 steps.  With the rescaled states the absorbing
    // row (possibly in the last lane) sums column n's (M + I) as its M at
    // column n + 1 into its Dh at column n + 2: every lane runs to column
    // n + 2 at least, so that this last term always takes the same FP32 path
    // whatever the other pairs of the tile (its M at the last step is then
    // exactly zero).
    const int total = HAT ? (nmax + P + 2) & ~1 : (nmax + P) & ~1;
    const char *ebase_lane = E + lane * 8;

    // Chain boundaries (wave-uniform).  Haplotype kc occupies stream
    // positions cpos .. cpos + nk - 1; lane t sweeps position s - t at step s.
    // At a boundary every lane clears its states before it sweeps a
    // position in [bA, bA + CW), bA = cpos + nk + 2: the columns before are
    // PAD, so M = I = 0 there in every real row (and every later M, I and D
    // is then exactly 0 until the next haplotype), and the absorbing row's D
    // holds the haplotype's whole sum, which the lane that holds it stores
    // (raw, converted by the epilogue).  Clearing steps are even steps CW
    // apart, each for the CW lanes whose window contains it; the first lane
    // of a group also takes the next haplotype's edge value.
    constexpr int CW = kChainSep - 2;
    static_assert(CW >= 2 && CW % 2 == 0, "clearing steps fall on even steps");
    int kc = 0, cpos = 0, nk = 0, bA = 0, rs_next = 0x7fffffff;
    if (chain && NH > 1) {
        nk = __builtin_amdgcn_readlane(nvec, 0);
        bA = nk + 2;
        rs_next = (bA + CW - 1) & ~1;
    }
    auto chain_clear = [&]() {
        const int lo = rs_next - bA - CW, hi = rs_next - bA;
        if (t > lo && t <= hi) {
            if (rml >= 0 && rml < K) {
                T dm = 0;
#pragma unroll
                for (int r = 0; r < K; ++r) dm = r == rml ? D[r] : dm;
                if constexpr (V)
                    acc = fmax(acc, (double)dm);
                else
                    acc += (double)dm;
                A.out_log10[rec.out + kc] = acc;
                acc = 0.0;
            }
#pragma unroll
            for (int r = 0; r < K; ++r) D[r] = 0;
            if (t == 0) {
                const T ne = (T)(e0f / (float)__builtin_amdgcn_readlane(nvec, kc + 1));
                if constexpr (P < 16) edge = ne;
                Xd = ne;
            }
        }
        if (hi >= P - 1) {
            // every lane of the group is past this boundary
            cpos += nk + kChainSep;
            ++kc;
            nk = __builtin_amdgcn_readlane(nvec, kc);
            if (kc < NH - 1) {
                bA = cpos + nk + 2;
                rs_next = (bA + CW - 1) & ~1;
            } else {
                rs_next = 0x7fffffff;
            }
        } else {
            rs_next += CW;
        }
    };

    for (int s0 = 0; s0 < total; s0 += CH) {
        uint32_t ahead[RingPer<P>::N];
        ring_load<P>(ahead, s0 / CH + 2, hap, nring, t);
        if constexpr (W) {
            // lane t stages the boundary row at column s0 + 1 + t, which
            // lane 0 takes at step s0 + t (zero in window 0: the row-0
            // boundary comes from `edge`)
            const int j = s0 + 1 + t;
            T v0 = 0, v1 = 0, v2 = 0;
            if (r0 > 0 && j <= n) {
                const T *b = bnd + (int64_t)j * 3;
                v0 = b[0];
                v1 = b[1];
                v2 = b[2];
            }
            top[t] = v0;
            top[64 + t] = v1;
            top[128 + t] = v2;
            __syncthreads();
        }
        const uint16_t *hp = ring + ((s0 - t) & (4 * CH - 1));
        const int cnt = min(CH, total - s0);
        T la[C::KP], lb[C::KP];
        load_lam<T, P, K>(la, ebase_lane + hp[0]);
        if constexpr (HAT) {
            // the steps of the chunk, in runs that end at a chain's clearing
            // steps (the run's loop has no branch of its own).  The ring reads
            // go through a volatile pointer: merged into one 32-bit read they
            // would be misaligned in every other lane.
            const volatile __attribute__((address_space(3))) uint16_t *hv =
                (const volatile __attribute__((address_space(3))) uint16_t *)hp;
            int u = 0;
            for (;;) {
                const int stop = (CHN && rs_next - s0 < cnt) ? rs_next - s0 : cnt;
                for (; u < stop; u += 2) {
                    load_lam<T, P, K>(lb, ebase_lane + hv[u + 1]);
                    if constexpr (W) {
                        window_step_hat<T, K, V>(M, I, D, Md, Id, Dd, la, ci, cd, ke, ep, edge, top, u, t, fin, bnd,
                                                 s0 + u, n);
                        load_lam<T, P, K>(la, ebase_lane + hv[u + 2]);
                        window_step_hat<T, K, V>(M, I, D, Md, Id, Dd, lb, ci, cd, ke, ep, edge, top, u + 1, t,
                                                 fin, bnd, s0 + u + 1, n);
                    } else {
                        cell_step_hx<T, P, K, V>(M, I, D, Xd, la, ci, cd, ke, ep, cib, cdb, keb, edge, keep);
                        load_lam<T, P, K>(la, ebase_lane + hv[u + 2]);
                        cell_step_hx<T, P, K, V>(M, I, D, Xd, lb, ci, cd, ke, ep, cib, cdb, keb, edge, keep);
                    }
                }
                if (u >= cnt) break;
                if constexpr (CHN) chain_clear();
            }
            // the absorbing row's Dh (Viterbi: its running maximum) moves
            // into the FP64 accumulator; nothing else reads it
            T dm = 0;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                dm = r == rml ? D[r] : dm;
                D[r] = r == rml ? (T)0 : D[r];
            }
            if constexpr (V)
                acc = fmax(acc, (double)dm);
            else
                acc += (double)dm;
        } else {
            T part = 0;
            for (int u = 0; u < cnt; u += 2) {
                load_lam<T, P, K>(lb, ebase_lane + hp[u + 1]);
                if constexpr (W) {
                    window_step<T, K, V>(M, I, D, Md, Id, Dd, la, al, be, de, ep, zt, epI0, edge, part, top, u, t,
                                         fin, bnd, s0 + u, n);
                    load_lam<T, P, K>(la, ebase_lane + hp[u + 2]);
                    window_step<T, K, V>(M, I, D, Md, Id, Dd, lb, al, be, de, ep, zt, epI0, edge, part, top, u + 1,
                                         t, fin, bnd, s0 + u + 1, n);
                } else {
                    cell_step<T, P, K, false, V>(M, I, D, Md, Id, Dd, la, al, be, de, ep, zt, epI0, edge, part);
                    load_lam<T, P, K>(la, ebase_lane + hp[u + 2]);
                    cell_step<T, P, K, false, V>(M, I, D, Md, Id, Dd, lb, al, be, de, ep, zt, epI0, edge, part);
                }
            }
            if constexpr (V)
                acc = fmax(acc, (double)part);
            else
                acc += (double)part;
        }
        ring_store<P>(ring, s0 / CH + 2, ahead, t, C::CODE_BYTES, chain);
        __syncthreads();
    }

    // ---- epilogue: the lane that holds the row-m sum writes it ---------------
    const bool owner = HAT ? (rml >= 0 && rml < K) : (t == P - 1);
    if constexpr (CHN) {
        if (chain) {
            // the last haplotype's raw sum joins the others; then the group's
            // lanes convert them, haplotype k in lane k mod P
            if (owner) A.out_log10[rec.out + NH - 1] = acc;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const int cls = m < 128 ? 0 : m < 256 ? 1 : m < 512 ? 2 : 3;
            for (int k = t; k < NH; k += P) {
                const int out = rec.out + k;
                const double sum = A.out_log10[out];
                A.out_log10[out] = log10(sum) - (double)kExp * 0.30102999566398119521;
                const bool ok = !gbad && (sum >= A.threshold) && (sum <= 3.0e38);
                if (!ok) {
                    // out of range: the rescaled FP64 sweep; a row outside the
                    // rescaled states (or the max-product score): the plain one
                    const int q = (gbad || V) ? kRescueClasses + cls : cls;
                    const int hk = h0 + k;
                    A.chain_recs[out] = PairRec{rec.read, hk, out, (int)(pb.hap_offset[hk + 1] - pb.hap_offset[hk])};
                    const int slot = atomicAdd(&A.book->rescue_count[q], 1);
                    A.rescue_list[q * A.rescue_stride + slot] = A.chain_rec_base + out;
                    if (A.out_status) A.out_status[out] = 1;  // final value written by the FP64 sweep
                } else if (A.out_status) {
                    A.out_status[out] = 0;
                }
            }
            return;
        }
    }
    if (gvalid && owner && fin) {
        const double lg = log10(acc) - (double)kExp * 0.30102999566398119521;
        const int cls = m < 128 ? 0 : m < 256 ? 1 : m < 512 ? 2 : 3;
        if (A.mode == kModeRescue && sizeof(T) == 8 && HAT) {
            // rescaled FP64 sweep: inside its range (and no row outside the
            // rescaled states), or passed on to the plain FP64 sweep
            if (!gbad && acc >= A.floor64 && acc <= 1.0e300) {
                A.out_log10[rec.out] = lg;
                if (A.out_status) A.out_status[rec.out] = 1;
            } else {
                const int q = kRescueClasses + cls;
                const int slot = atomicAdd(&A.book->rescue_count[q], 1);
                A.rescue_list[q * A.rescue_stride + slot] = ridx;
                atomicAdd(&A.book->rescue_passed, 1);
            }
        } else if (A.mode == kModeRescue) {
            A.out_log10[rec.out] = lg;
            if (A.out_status) A.out_status[rec.out] = (acc >= A.floor64) ? 1 : 2;
        } else {
            A.out_log10[rec.out] = lg;
            const bool ok = !gbad && (acc >= A.threshold) && (acc <= 3.0e38);
            if (A.mode == kModeBinned && !ok) {
                if (W) {
                    const int slot = atomicAdd(&A.book->long_rescue_count, 1);
                    A.long_rescue_list[slot] = ridx;
                } else {
                    // out of range: the rescaled FP64 sweep; a row outside the
                    // rescaled states (or the max-product score): the plain one
                    const int q = (gbad || V) ? kRescueClasses + cls : cls;
                    const int slot = atomicAdd(&A.book->rescue_count[q], 1);
                    A.rescue_list[q * A.rescue_stride + slot] = ridx;
                }
                if (A.out_status) A.out_status[rec.out] = 1;  // final value written by the FP64 sweep
            } else if (A.out_status) {
                A.out_status[rec.out] = ok ? 0 : 3;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// compiled configurations of the FP32 sweep (lanes per pair, rows per lane)
// ---------------------------------------------------------------------------
#define PH_FWD32_CONFIGS(X) \
    X(4, 2) X(4, 3) X(4, 4) X(4, 5) X(4, 6) X(4, 7) X(4, 8) X(4, 9) X(4, 10) X(4, 11) X(4, 12) \
    X(4, 13) X(4, 14) X(4, 15) X(4, 16) \
    X(8, 2) X(8, 3) X(8, 4) X(8, 5) X(8, 6) X(8, 7) X(8, 8) X(8, 9) X(8, 10) X(8, 11) X(8, 12) \
    X(8, 13) X(8, 14) X(8, 15) X(8, 16) \
    X(16, 1) X(16, 2) X(16, 3) X(16, 4) X(16, 5) X(16, 6) X(16, 7) X(16, 8) \
    X(16, 9) X(16, 10) X(16, 11) X(16, 12) X(16, 13) X(16, 14) X(16, 15) X(16, 16) \
    X(32, 4) X(32, 6) X(32, 8) X(32, 10) X(32, 12) X(32, 16) \
    X(64, 2) X(64, 3) X(64, 4) X(64, 5) X(64, 6) X(64, 7) X(64, 8) X(64, 9) X(64, 10) \
    X(64, 11) X(64, 12) X(64, 13) X(64, 14) X(64, 15) X(64, 16)

bool fwd32_supported(int P, int K)
{
#define PH_SUP(p, k) if (P == p && K == k) return true;
    PH_FWD32_CONFIGS(PH_SUP)
#undef PH_SUP
    return false;
}

// Persistent FP32 sweep over the tiles of one length bin: every wave takes
// the next tile (one read/haplotype pair per lane group) from the bin's
// cursor.  Records of a bin are ordered longest haplotype first.
// waves per SIMD each configuration should reach (register budget 512 / W)
#ifndef PH_W4_MAX_K
#define PH_W4_MAX_K 6
#endif
#ifndef PH_W3_MAX_K
#define PH_W3_MAX_K 10
#endif
constexpr int waves_for(int K) { return K <= PH_W4_MAX_K ? 4 : K <= PH_W3_MAX_K ? 3 : 2; }
// the max-product cell keeps more temporaries live (no FMA contraction)
constexpr int waves_for_viterbi(int K) { return K <= 5 ? 4 : K <= 8 ? 3 : 2; }

template <int P, int K, bool V = false>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(V ? waves_for_viterbi(K) : waves_for(K)))) void k_fwd32(SweepArgs A, int bin)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<float, P, K>::LDS_BYTES];
    Book *bk = A.book;
    constexpr int G = 64 / P;
    const int rb = bk->bin_rec_begin[bin], re = bk->bin_rec_begin[bin + 1];
    const int ntiles = (re - rb + G - 1) / G;
    int tile = next_tile(&bk->bin_counter[bin]);
    while (tile < ntiles) {
        const int first = rb + tile * G;
        sweep_tile<float, P, K, false, V>(A, nullptr, first, min(G, re - first), lds);
        tile = next_tile(&bk->bin_counter[bin]);
    }
}

// One persistent FP32 launch over every length bin of 16-lane groups with
// K = 3..16 rows per lane (reads up to 255 bases): the wave takes the next
// tile from one cursor and dispatches on the tile's bin.  Bins are laid out
// longest first, so waves drain the long tiles first.  (Configurations with
// other lane counts run as one launch per bin.)
#define PH_SINGLE_CONFIGS(X) \
    X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_fwd32_single(SweepArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<float, 16, 16>::LDS_BYTES];
    Book *bk = A.book;
    const int ntiles = bk->bin_tile_begin[A.num_bins];
    int tile = next_tile(&bk->tile_counter);
    while (tile < ntiles) {
        int b = 0;
        while (tile >= bk->bin_tile_begin[b + 1]) ++b;
        constexpr int G = 4;
        const int first = bk->bin_rec_begin[b] + (tile - bk->bin_tile_begin[b]) * G;
        const int nvalid = min(G, bk->bin_rec_begin[b + 1] - first);
        switch (A.bins[b].K) {
#define PH_SC(k) \
    case k: sweep_tile<float, 16, k>(A, nullptr, first, nvalid, lds); break;
            PH_SINGLE_CONFIGS(PH_SC)
#undef PH_SC
        default: break;
        }
        tile = next_tile(&bk->tile_counter);
    }
}

bool single_supported(int P, int K) { return P == 16 && K >= 3 && K <= 16; }

// Plain FP32 sweep: one pair per wave, pairs in output order, one (64, K).
template <int K>
__global__ __launch_bounds__(64) void k_plain32(SweepArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<float, 64, K>::LDS_BYTES];
    int tile = next_tile(&A.book->tile_counter);
    while (tile < A.plain_count) {
        sweep_tile<float, 64, K>(A, nullptr, tile, 1, lds);
        tile = next_tile(&A.book->tile_counter);
    }
}

// FP64 sweep over one rescue queue (64 lanes per pair, K rows per lane):
// H = true, the rescaled states over the pairs that left the FP32 range;
// H = false, the plain states over the second set of queues.
template <int K, bool V = false, bool H = false>
__global__ __launch_bounds__(64) void k_fwd64(SweepArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<double, 64, K>::LDS_BYTES];
    const int q = (H ? 0 : kRescueClasses) + A.rescue_class;
    const int count = A.book->rescue_count[q];
    const int32_t *list = A.rescue_list + q * A.rescue_stride;
    int tile = next_tile(&A.book->rescue_counter[q]);
    while (tile < count) {
        sweep_tile<double, 64, K, false, V, H>(A, list, tile, 1, lds);
        tile = next_tile(&A.book->rescue_counter[q]);
    }
}

// Windowed sweeps of reads longer than kMaxReadLen: one launch per window of
// kLongRows rows, in window order on one stream.  FP32: the tiles of the
// long bin (one pair each, slot = position in the bin); FP64: the long-pair
// rescue queue (slot = queue position).  A pair whose rows end in an earlier
// window is skipped.
template <bool V>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_long32(SweepArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<float, 64, 16>::LDS_BYTES + 3 * 64 * sizeof(float)];
    Book *bk = A.book;
    const int rb = bk->bin_rec_begin[A.long_bin], re = bk->bin_rec_begin[A.long_bin + 1];
    int tile = next_tile(&bk->long_counter[A.window]);
    while (tile < re - rb) {
        sweep_tile<float, 64, 16, true, V>(A, nullptr, rb + tile, 1, lds, tile);
        tile = next_tile(&bk->long_counter[A.window]);
    }
}

template <bool V>
__global__ __launch_bounds__(64) void k_long64(SweepArgs A)
{
    __shared__ __attribute__((aligned(16))) char lds[Cfg<double, 64, 16>::LDS_BYTES + 3 * 64 * sizeof(double)];
    Book *bk = A.book;
    const int count = bk->long_rescue_count;
    int item = next_tile(&bk->long64_counter[A.window]);
    while (item < count) {
        sweep_tile<double, 64, 16, true, V>(A, A.long_rescue_list, item, 1, lds, item);
        item = next_tile(&bk->long64_counter[A.window]);
    }
}

// ---------------------------------------------------------------------------
// binning: counting sort of the pairs by (length bin, haplotype-length bucket)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pair_key(const BinArgs &a, int64_t k, PairRec &rec)
{
    int lo = 0, hi = a.num_batches;  // largest q with out_offset[q] <= k
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.out_offset[mid] <= k) lo = mid; else hi = mid;
    }
    const int q = lo;
    const int local = (int)(k - a.out_offset[q]);
    const int nh = a.batch_hap_begin[q + 1] - a.batch_hap_begin[q];
    const int r = a.batch_read_begin[q] + local / nh;
    const int h = a.batch_hap_begin[q] + local % nh;
    const int m = (int)(a.read_offset[r + 1] - a.read_offset[r]);
    const int n = (int)(a.hap_offset[h + 1] - a.hap_offset[h]);
    rec.read = r;
    rec.hap = h;
    rec.out = (int)k;
    rec.n = n;
    int b = a.m2bin[m > kMaxReadLen ? kMaxReadLen + 1 : m];
    const int nb = n < 1024 ? (n >> 4) : 64 + min((n - 1024) >> 7, 63);
    if (a.split && nb >= a.split[b]) b = a.split[kMaxBins + b];
    return b * kBuckets + (kBuckets - 1 - nb);
}

__global__ __launch_bounds__(256) void k_reset(int32_t *hist, int nkeys, Book *bk)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < nkeys; i += gridDim.x * 256) hist[i] = 0;
    if (blockIdx.x == 0) {
        int32_t *w = (int32_t *)bk;
        for (int i = threadIdx.x; i < (int)(sizeof(Book) / 4); i += 256) w[i] = 0;
    }
}

__global__ __launch_bounds__(256) void k_bin_count(BinArgs a)
{
    __shared__ int h[kMaxKeys];
    const int nk = a.num_bins * kBuckets;
    for (int i = threadIdx.x; i < nk; i += 256) h[i] = 0;
    __syncthreads();
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < a.num_pairs;
         k += (int64_t)gridDim.x * 256) {
        PairRec rec;
        atomicAdd(&h[pair_key(a, k, rec)], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nk; i += 256)
        if (h[i]) atomicAdd(&a.hist[i], h[i]);
}

// Set-up of the plan-free forward (ph_forward_batch_noalloc), one block:
// the output offset of every batch (exclusive scan of |R_q| |H_q|), the
// read-length -> bin map and the pairs per tile of every bin, which a plan
// computes on the host and uploads once.
__global__ __launch_bounds__(1024) void k_na_setup(const int32_t *rb, const int32_t *hb, int32_t nb,
                                                   int64_t *out_offset, int16_t *m2bin, int32_t *bin_G,
                                                   BinTable t)
{
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    for (int m = tid; m <= kMaxReadLen + 1; m += 1024) {
        int e = 0;
        while (e < t.num_bins - 1 && t.max_m[e] < m) ++e;
        m2bin[m] = (int16_t)(t.num_bins - 1 - e);
    }
    if (tid < t.num_bins) bin_G[tid] = 64 / t.P[t.num_bins - 1 - tid];
    const int per = (nb + 1023) / 1024;
    const int q0 = min(tid * per, nb), q1 = min(q0 + per, nb);
    int64_t sum = 0;
    for (int q = q0; q < q1; ++q) sum += (int64_t)(rb[q + 1] - rb[q]) * (hb[q + 1] - hb[q]);
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int q = q0; q < q1; ++q) {
        out_offset[q] = run;
        run += (int64_t)(rb[q + 1] - rb[q]) * (hb[q + 1] - hb[q]);
    }
    if (tid == 1023) out_offset[nb] = part[1023];
}

// one block: exclusive scan of the key histogram (in place, becomes the
// scatter cursors), record and tile ranges of every bin.
__global__ __launch_bounds__(1024) void k_bin_scan(BinArgs a)
{
    __shared__ int part[1024];
    const int nk = a.num_bins * kBuckets;
    constexpr int PER = kMaxKeys / 1024;
    int loc[PER];
    int sum = 0;
    for (int j = 0; j < PER; ++j) {
        int i = threadIdx.x * PER + j;
        loc[j] = i < nk ? a.hist[i] : 0;
        sum += loc[j];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - sum;
    for (int j = 0; j < PER; ++j) {
        int i = threadIdx.x * PER + j;
        if (i < nk) {
            a.hist[i] = run;
            if (i % kBuckets == 0) a.book->bin_rec_begin[i / kBuckets] = run;
        }
        run += loc[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Book *bk = a.book;
        bk->bin_rec_begin[a.num_bins] = (int)a.num_pairs;
        int tiles = 0;
        for (int b = 0; b < a.num_bins; ++b) {
            bk->bin_tile_begin[b] = tiles;
            const int cnt = bk->bin_rec_begin[b + 1] - bk->bin_rec_begin[b];
            const int G = a.bin_G[b];
            tiles += (cnt + G - 1) / G;
        }
        bk->bin_tile_begin[a.num_bins] = tiles;
    }
}

constexpr int kScatterPer = 8;  // pairs per thread in the scatter

__global__ __launch_bounds__(256) void k_bin_scatter(BinArgs a)
{
    __shared__ int cnt[kMaxKeys];
    __shared__ int base[kMaxKeys];
    const int nk = a.num_bins * kBuckets;
    for (int i = threadIdx.x; i < nk; i += 256) cnt[i] = 0;
    __syncthreads();
    PairRec rec[kScatterPer];
    int key[kScatterPer], rank[kScatterPer];
    const int64_t first = (int64_t)blockIdx.x * 256 * kScatterPer;
    for (int j = 0; j < kScatterPer; ++j) {
        int64_t k = first + (int64_t)j * 256 + threadIdx.x;
        key[j] = -1;
        if (k < a.num_pairs) {
            key[j] = pair_key(a, k, rec[j]);
            rank[j] = atomicAdd(&cnt[key[j]], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nk; i += 256)
        if (cnt[i]) base[i] = atomicAdd(&a.hist[i], cnt[i]);
    __syncthreads();
    for (int j = 0; j < kScatterPer; ++j)
        if (key[j] >= 0) a.recs[base[key[j]] + rank[j]] = rec[j];
}

// The book of a plan whose work lists were built at plan creation: bin
// ranges from the plan's image, every cursor and queue length zero.
__global__ __launch_bounds__(256) void k_book_copy(Book *bk, const Book *img)
{
    int32_t *w = (int32_t *)bk;
    const int32_t *r = (const int32_t *)img;
    for (int i = threadIdx.x; i < (int)(sizeof(Book) / 4); i += 256) w[i] = r[i];
}

// Chain code stream: haplotype h at hap_offset[h] + kChainSep h, its base
// codes (above 4: N) followed by kChainSep PAD codes.  One wave per haplotype.
__global__ __launch_bounds__(256) void k_chain_codes(const int64_t *ho, const uint8_t *hb, int32_t nh,
                                                     uint8_t *codes)
{
    const int lane = threadIdx.x & 63;
    for (int h = blockIdx.x * 4 + (threadIdx.x >> 6); h < nh; h += gridDim.x * 4) {
        const int64_t a = ho[h], n = ho[h + 1] - a;
        uint8_t *dst = codes + a + (int64_t)kChainSep * h;
        for (int64_t i = lane; i < n + kChainSep; i += 64)
            dst[i] = i < n ? (uint8_t)clamp_code(hb[a + i]) : (uint8_t)kPad;
    }
}

__global__ __launch_bounds__(256) void k_plain_records(BinArgs a)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < a.num_pairs;
         k += (int64_t)gridDim.x * 256) {
        PairRec rec;
        pair_key(a, k, rec);
        a.recs[k] = rec;
    }
}

// Explicit-parameter mode: exponentiate the log10 parameters of every read
// position once per call, [npos][7] float -> [npos][8] double.
__global__ __launch_bounds__(256) void k_prep_params(const float *lg, int64_t npos, double *lin)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npos * 8;
         i += (int64_t)gridDim.x * 256) {
        const int64_t pos = i >> 3;
        const int c = (int)(i & 7);
        lin[i] = c < 7 ? exp10((double)lg[pos * 7 + c]) : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_validate(const uint8_t *rb, int64_t nr, const uint8_t *hb,
                                                  int64_t nh, int32_t *bad_count)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nr; i += (int64_t)gridDim.x * 256)
        bad += rb[i] > 4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nh; i += (int64_t)gridDim.x * 256)
        bad += hb[i] > 4;
    if (bad) atomicAdd(bad_count, bad);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int occupancy(const void *fn);

static int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_bin_count(const BinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(a.num_pairs, 256 * 16, 2048)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const BinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const BinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(a.num_pairs, 256 * kScatterPer, 1 << 30)),
                       dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_plain_records(const BinArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_plain_records, dim3(grid_for(a.num_pairs, 256 * 4, 4096)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reset_keys(int32_t *hist, int nkeys, Book *book, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(grid_for(nkeys, 256, 64)), dim3(256), 0, s, hist, nkeys, book);
    return hipGetLastError();
}

hipError_t launch_book_copy(Book *book, const Book *image, hipStream_t s)
{
    hipLaunchKernelGGL(k_book_copy, dim3(1), dim3(256), 0, s, book, image);
    return hipGetLastError();
}

hipError_t launch_chain_codes(const int64_t *hap_offset, const uint8_t *hap_bases, int32_t num_haps,
                              uint8_t *codes, hipStream_t s)
{
    hipLaunchKernelGGL(k_chain_codes, dim3(grid_for(num_haps, 4, 4096)), dim3(256), 0, s, hap_offset, hap_bases,
                       num_haps, codes);
    return hipGetLastError();
}

hipError_t launch_fwd32(const SweepArgs &a_in, int P, int K, int bin, int grid, hipStream_t s)
{
    SweepArgs a = a_in;
    a.mode = kModeBinned;
#define PH_L32(p, k)                                                                        \
    if (P == p && K == k) {                                                                 \
        if (a.viterbi)                                                                      \
            hipLaunchKernelGGL((k_fwd32<p, k, true>), dim3(grid), dim3(64), 0, s, a, bin);  \
        else                                                                                \
            hipLaunchKernelGGL((k_fwd32<p, k, false>), dim3(grid), dim3(64), 0, s, a, bin); \
        return hipGetLastError();                                                           \
    }
    PH_FWD32_CONFIGS(PH_L32)
#undef PH_L32
    return hipErrorInvalidValue;
}

hipError_t launch_fwd32_single(const SweepArgs &a_in, int grid, hipStream_t s)
{
    SweepArgs a = a_in;
    a.mode = kModeBinned;
    hipLaunchKernelGGL(k_fwd32_single, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

int fwd32_single_blocks_per_cu() { return occupancy((const void *)k_fwd32_single); }

hipError_t launch_plain32(const SweepArgs &a_in, int K, int grid, hipStream_t s)
{
    SweepArgs a = a_in;
    a.mode = kModePlain;
    switch (K) {
#define PH_PK(k) case k: hipLaunchKernelGGL(k_plain32<k>, dim3(grid), dim3(64), 0, s, a); break;
        PH_PK(1) PH_PK(2) PH_PK(3) PH_PK(4) PH_PK(5) PH_PK(6) PH_PK(7) PH_PK(8)
        PH_PK(9) PH_PK(10) PH_PK(11) PH_PK(12) PH_PK(13) PH_PK(14) PH_PK(15) PH_PK(16)
#undef PH_PK
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static const int kRescueK[kRescueClasses] = {2, 4, 8, 16};

hipError_t launch_fwd64(const SweepArgs &a, int cls, bool rescaled, int grid, hipStream_t s)
{
    SweepArgs b = a;
    b.rescue_class = cls;
    b.mode = kModeRescue;
    if (b.viterbi && rescaled) return hipSuccess;  // the max-product score uses the plain queues only
#define PH_L64(k)                                                                            \
    case k:                                                                                  \
        if (b.viterbi)                                                                       \
            hipLaunchKernelGGL((k_fwd64<k, true, false>), dim3(grid), dim3(64), 0, s, b);    \
        else if (rescaled)                                                                   \
            hipLaunchKernelGGL((k_fwd64<k, false, true>), dim3(grid), dim3(64), 0, s, b);    \
        else                                                                                 \
            hipLaunchKernelGGL((k_fwd64<k, false, false>), dim3(grid), dim3(64), 0, s, b);   \
        break;
    switch (kRescueK[cls]) {
        PH_L64(2) PH_L64(4) PH_L64(8) PH_L64(16)
    default: return hipErrorInvalidValue;
    }
#undef PH_L64
    return hipGetLastError();
}

hipError_t launch_long32(const SweepArgs &a, int window, int grid, hipStream_t s)
{
    SweepArgs b = a;
    b.window = window;
    b.mode = kModeBinned;
    if (b.viterbi)
        hipLaunchKernelGGL(k_long32<true>, dim3(grid), dim3(64), 0, s, b);
    else
        hipLaunchKernelGGL(k_long32<false>, dim3(grid), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_long64(const SweepArgs &a, int window, int grid, hipStream_t s)
{
    SweepArgs b = a;
    b.window = window;
    b.mode = kModeRescue;
    if (b.viterbi)
        hipLaunchKernelGGL(k_long64<true>, dim3(grid), dim3(64), 0, s, b);
    else
        hipLaunchKernelGGL(k_long64<false>, dim3(grid), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_na_setup(const int32_t *rb, const int32_t *hb, int32_t nb, int64_t *out_offset,
                           int16_t *m2bin, int32_t *bin_G, const BinTable &t, hipStream_t s)
{
    hipLaunchKernelGGL(k_na_setup, dim3(1), dim3(1024), 0, s, rb, hb, nb, out_offset, m2bin, bin_G, t);
    return hipGetLastError();
}

hipError_t launch_prep_params(const float *lg, int64_t npos, double *lin, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep_params, dim3(grid_for(npos * 8, 256 * 4, 8192)), dim3(256), 0, s, lg,
                       npos, lin);
    return hipGetLastError();
}

hipError_t launch_validate(const DevProblem &pb, int64_t nrb, int64_t nhb, int32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate, dim3(grid_for(nrb + nhb, 256 * 8, 4096)), dim3(256), 0, s,
                       pb.read_bases, nrb, pb.hap_bases, nhb, bad);
    return hipGetLastError();
}

static int occupancy(const void *fn)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

int fwd32_blocks_per_cu(int P, int K)
{
#define PH_O32(p, k) if (P == p && K == k) return occupancy((const void *)k_fwd32<p, k>);
    PH_FWD32_CONFIGS(PH_O32)
#undef PH_O32
    return 1;
}

int plain32_blocks_per_cu(int K)
{
    switch (K) {
#define PH_PO(k) case k: return occupancy((const void *)k_plain32<k>);
        PH_PO(1) PH_PO(2) PH_PO(3) PH_PO(4) PH_PO(5) PH_PO(6) PH_PO(7) PH_PO(8)
        PH_PO(9) PH_PO(10) PH_PO(11) PH_PO(12) PH_PO(13) PH_PO(14) PH_PO(15) PH_PO(16)
#undef PH_PO
    }
    return 1;
}

int long32_blocks_per_cu() { return occupancy((const void *)k_long32<false>); }
int long64_blocks_per_cu() { return occupancy((const void *)k_long64<false>); }

int fwd64_blocks_per_cu(int cls, bool rescaled)
{
    switch (kRescueK[cls]) {
    case 2: return occupancy(rescaled ? (const void *)k_fwd64<2, false, true> : (const void *)k_fwd64<2>);
    case 4: return occupancy(rescaled ? (const void *)k_fwd64<4, false, true> : (const void *)k_fwd64<4>);
    case 8: return occupancy(rescaled ? (const void *)k_fwd64<8, false, true> : (const void *)k_fwd64<8>);
    case 16: return occupancy(rescaled ? (const void *)k_fwd64<16, false, true> : (const void *)k_fwd64<16>);
    }
    return 1;
}

}  // namespace ph
