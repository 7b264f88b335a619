// Adjoint (backward) of the Pair-HMM forward algorithm on gfx950.
//
// The paper computes only the forward likelihood (arXiv 2411.11547,
// Section II-A, Eq. 1-4).  Its derivatives follow from the same DP run
// backwards.  The FP32 pass carries the forward sweep's rescaled states
// (M, Ih, Dh), whose recurrences and reverse recurrences are given with
// adj_backward below; the FP64 pass carries (M, I, D') with D' = beta_{i+1} D,
// D' = zeta'_i M(i,j-1) + eps_i D'(i,j-1), zeta'_i = beta_{i+1} zeta_i, so
// that M(i,j) = lam_ij (alpha_i M + beta_i I + D')(i-1,j-1).  With
// B_X(i,j) = dL/dX(i,j) and B(m,.) seeded by the result formula
// L = sum_j M(m,j) + I(m,j), every term sends its coefficient back to its
// source cell,
//
//   B_M(i,j)  = alpha_{i+1} Bl(i+1,j+1) + delta_{i+1} B_I(i+1,j) + zeta'_i B_D'(i,j+1)
//   B_I(i,j)  = beta_{i+1}  Bl(i+1,j+1) + eps_{i+1}  B_I(i+1,j)
//   B_D'(i,j) =             Bl(i+1,j+1) + eps_i      B_D'(i,j+1)
//   Bl(i,j)   = lam_ij B_M(i,j)
//
// and d log10 L / d log10 theta_i (the posterior expected number of uses of
// theta_i) is a sum over row i of forward value x coefficient x backward
// value, divided by L: beta_i's sum is over (beta_i I + D')(i-1,j-1) Bl(i,j)
// (D' of row i-1 carries beta_i), zeta_i's over zeta'_i M(i,j-1) B_D'(i,j),
// and eps_i's D part over eps_i D'(i,j-1) B_D'(i,j), the two betas cancelling.
//
// Layout: the lane structure of the forward sweep (P lanes per pair, K rows
// per lane, lane t at column j = s - t + 1 of step s).  Memory is bounded by
// checkpoints: every CB steps each lane stores its K-row state and the three
// diagonal values it holds from the lane above, 3K + 3 values per lane.  The
// backward walks the blocks of CB steps in reverse: the wave reloads a
// block's checkpoint, recomputes the block's CB steps as a wavefront (the
// same lane exchange as the forward, so nothing else needs storing), keeps
// them in registers and runs the reverse wavefront over them.  In the FP32
// pass the memory unit copies the next block's checkpoint into LDS while the
// current block runs (global_load_lds), so the reload costs neither
// registers nor a wait on memory.
//
// One persistent workgroup per slot takes a tile (G = 64/P pairs of one
// (P, K) configuration), runs the checkpointed forward into its own slice of
// the workspace and then the reverse sweep; the slice is read back soon after
// it is written, in reverse order, and waves in the forward phase (stores)
// overlap waves in the reverse phase (arithmetic).  Each pair writes its own
// gradient rows (a read's rows directly when it has one pair, else rows of a
// per-pair array that a fixed-order sum over the read's pairs reduces), so
// no float atomics are needed and results do not depend on timing.
//
// Precision (the forward's FP32 sweep with FP64 recomputation, carried over
// to the adjoint): an FP32 pass handles every pair; a pair whose scaled FP32
// sum leaves the FP32 range is queued by read-length class and redone by an
// FP64 pass (64 lanes per pair, one pair at a time per workgroup).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ph_device.h"
#include "ph_internal.h"

// 1: the reverse sweep prefetches the next block's checkpoint into registers
// (configurations where that does not spill)
#ifndef PH_ADJ_PREFETCH
#define PH_ADJ_PREFETCH 1
#endif

namespace ph {

__constant__ double c_prob[256];  // Phred q -> 10^(-q/10), computed on the host in FP64

hipError_t upload_luts_adjoint()
{
    double t[256];
    for (int q = 0; q < 256; ++q) t[q] = pow(10.0, -(double)q / 10.0);
    return hipMemcpyToSymbol(HIP_SYMBOL(c_prob), t, sizeof(t));
}

// Lane t receives lane t+1's value inside 16-lane rows (P = 16) or across
// the wave (P = 32, 64); only the wave's last lane (row's, for P = 16)
// receives 0, so the last lane of a 32-lane group holds the next group's
// first lane and callers scale it away.
template <int P>
__device__ __forceinline__ uint32_t shift_down_raw_u(uint32_t v)
{
    int x = (int)v;
    if constexpr (P == 16)
        x = __builtin_amdgcn_mov_dpp(x, 0x101 /* row_shl:1 */, 0xf, 0xf, true);
    else
        x = __builtin_amdgcn_mov_dpp(x, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
    return (uint32_t)x;
}

template <int P>
__device__ __forceinline__ float shift_down_raw(float v)
{
    return __builtin_bit_cast(float, shift_down_raw_u<P>(__builtin_bit_cast(uint32_t, v)));
}

template <int P>
__device__ __forceinline__ double shift_down_raw(double v)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = shift_down_raw_u<P>((uint32_t)u);
    uint32_t hi = shift_down_raw_u<P>((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Scaling of the two precisions.  The forward starts from D(0,j) = 2^kFwd / n.
// The backward is seeded with B(m,.) = 2^(kProd - ilogb(L_s)), L_s the scaled
// likelihood: every product F(i,j) B(i,j) counts path mass through one cell,
// so it stays below about 2^kProd, and B itself stays below 2^SB (the
// continuation mass of a cell is at most 1), which the range floor of each
// precision keeps finite.
template <typename T>
struct AdjRange;
template <>
struct AdjRange<float> {
    static constexpr int kFwd = 120, kProd = 30;
};
template <>
struct AdjRange<double> {
    static constexpr int kFwd = 1020, kProd = 20;
};

template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
    using V = float2;
};
template <>
struct Pair2<double> {
    using V = double2;
};

template <typename T, int P, int K>
struct AdjCfg {
    static constexpr int G = 64 / P;
    // E[code][row][lane] = lam, negated where the row's base mismatches the
    // code (the sign carries the mismatch flag; every lam is >= 0)
    static constexpr int ENT = (int)sizeof(T);
    static constexpr int ROW_BYTES = 64 * ENT;
    static constexpr int CODE_BYTES = K * ROW_BYTES;
    static constexpr int E_BYTES = kCodes * CODE_BYTES;
};

// Per-pair state shared by the forward and backward parts: the record, the
// per-row coefficients of the lane's K rows (absorbing rows past the read end,
// as in the forward sweep), the emission table with mismatches marked by the
// sign, and the haplotype's codes staged in LDS with PAD outside columns
// 1..n.
//
// FP32 (HAT): the forward's rescaled states Ih = beta_{i+1} I and
// Dh = D / zeta_i, with al = alpha, cd = beta_i zeta_{i-1}, kd = beta_{i+1}
// delta_i, ke = beta_{i+1} eps_i / beta_i, ep = eps (beta after the last read
// row read as 1; the read's first row has al = cd = kd = ke = 0, its boundary
// D entering as the edge value through Ih).  The absorbing row m + 1 has
// lam = al = ep = 1 and sums the last read row's M + I along its Dh; rows
// past it are zero.  A row with beta below 2^-20 sends the pair to FP64.
// FP64: D carried as D' = beta_{i+1} D, al, be, de, ep as Eq. (1)-(3) and
// ze = beta_{i+1} zeta_i, the absorbing rows passing I down to the group's
// last lane.
template <typename T, int P, int K>
struct AdjPair {
    static constexpr bool HAT = sizeof(T) == 4;
    using C = AdjCfg<T, P, K>;
    using V2 = typename Pair2<T>::V;
    int lane, g, t;
    AdjRec rec;
    int64_t ro;
    int m, n, S;
    int rml;     // the absorbing row's index among the lane's rows (HAT; out of 0..K-1 elsewhere)
    bool bad;    // HAT: one of the lane's rows has beta below 2^-20
    T edge;      // the read's first row's boundary D (scaled), first lane only
    T al[K], be[K], de[K], ep[K], ze[K];  // plain states (be, de, ze unused with HAT)
    T cd[K], kd[K], ke[K];                // rescaled states
    char *E;
    const char *El;      // the lane's column of the emission table
    const uint8_t *hs;   // staged haplotype codes (PAD outside 1..n); column j at hs[j + P]
    T *ckl;              // FP32: the wave's LDS checkpoint buffer [3K+3][64], after the staged haplotypes

    // The lane's K rows, rescaled states: coefficients into registers and
    // emissions into the lane's column of the table.  The quality bytes of
    // the K rows (and of the rows on either side) are all requested before
    // any is used, so the tile waits for memory once, not once per row.
    __device__ __forceinline__ void init_rows_hat(const AdjArgs &A, char *mine)
    {
        const DevProblem &pb = A.pb;
        const double *L = A.lin_params;
        // Phred mode: the quality bytes of rows base-1 .. base+K, all loads
        // issued at once; the table lookups that follow hit the cache
        uint32_t qb[K], qi[K], qd[K], qg[K], qgn[K], qdp[K], code[K];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int i = t * K + r;
            const int64_t pos = ro + min(i, m - 1);
            code[r] = pb.read_bases[pos];
            if (!L) {
                qb[r] = pb.bq[pos];
                qi[r] = pb.iq[pos];
                qd[r] = pb.dq[pos];
                qg[r] = pb.gq[pos];
                qgn[r] = pb.gq[ro + min(i + 1, m - 1)];
                qdp[r] = pb.dq[ro + max(min(i - 1, m - 1), 0)];
            }
        }
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int i = t * K + r;
            const int64_t pos = ro + min(i, m - 1);
            double pa, pbt, pd, pe, plm, plx, bnx, zpv;
            if (L) {
                const double *q = L + pos * 8;
                pa = q[0];
                pbt = q[1];
                pd = q[2];
                pe = q[3];
                plm = q[5];
                plx = q[6];
                bnx = L[(ro + min(i + 1, m - 1)) * 8 + 1];
                zpv = L[(ro + max(min(i - 1, m - 1), 0)) * 8 + 4];
            } else {
                const double Q = c_prob[qb[r]];
                pd = c_prob[qi[r]];
                const double z = c_prob[qd[r]];
                pe = c_prob[qg[r]];
                pa = 1.0 - pd - z;
                pbt = 1.0 - pe;
                plm = 1.0 - Q;
                plx = Q / 3.0;
                bnx = 1.0 - c_prob[qgn[r]];
                zpv = c_prob[qdp[r]];
            }
            const bool real = i < m;
            const bool inner = real && i >= 1;
            const double bn = (i + 1 < m) ? bnx : 1.0;
            const double zp = inner ? zpv : 0.0;
            const bool ok = pbt >= 0x1p-20;
            bad = bad || (inner && !ok);
            al[r] = i == 0 ? (T)0 : real ? (T)pa : (i == m ? (T)1 : (T)0);
            cd[r] = inner ? (T)(pbt * zp) : (T)0;
            kd[r] = inner ? (T)(bn * pd) : (T)0;
            ke[r] = (inner && ok) ? (T)(bn * pe / pbt) : (T)0;
            ep[r] = real ? (T)pe : (i == m ? (T)1 : (T)0);
            const bool one = i == m;  // the absorbing row takes every column with lam = 1
            const uint32_t cr = clamp_code(code[r]);
#pragma unroll
            for (int c = 0; c < kCodes; ++c) {
                const bool match = cr == (uint32_t)c || cr == 4u || c == 4;
                T v = one ? (T)1 : (T)0;
                if (real && c != kPad) v = match ? (T)plm : -(T)plx;
                *(T *)(mine + c * C::CODE_BYTES + r * C::ROW_BYTES) = v;
            }
        }
    }

    // The same for the plain states of the FP64 pass, one row at a time (the
    // row parameters parked in the lane's own table entries, then loaded).
    __device__ __forceinline__ void init_rows_plain(const AdjArgs &A, char *mine)
    {
        const DevProblem &pb = A.pb;
        auto slot = [&](int c, int r) -> T * { return (T *)(mine + c * C::CODE_BYTES + r * C::ROW_BYTES); };
#pragma unroll 1
        for (int r = 0; r < K; ++r) {
            const int i = t * K + r;
            const int ic = min(i, m - 1);
            const RowPar p = load_row(pb, A.lin_params, ro + ic, c_prob);
            const bool real = i < m;
            *slot(0, r) = real ? (T)p.a : (T)0;
            *slot(1, r) = real ? (T)p.b : (T)0;
            *slot(2, r) = real ? (T)p.d : (i == m ? (T)1 : (T)0);
            *slot(3, r) = real ? (T)p.e : (T)1;
            const double bnext = (i + 1 < m) ? load_beta(pb, A.lin_params, ro + i + 1, c_prob) : 0.0;
            *slot(4, r) = real ? (T)(p.z * bnext) : (T)0;
        }
#pragma unroll
        for (int r = 0; r < K; ++r) {
            al[r] = *slot(0, r);
            be[r] = *slot(1, r);
            de[r] = *slot(2, r);
            ep[r] = *slot(3, r);
            ze[r] = *slot(4, r);
        }
#pragma unroll 1
        for (int r = 0; r < K; ++r) {
            const int i = t * K + r;
            const int ic = min(i, m - 1);
            const RowPar p = load_row(pb, A.lin_params, ro + ic, c_prob);
            const bool real = i < m;
            const uint32_t code = clamp_code(pb.read_bases[ro + ic]);
#pragma unroll
            for (int c = 0; c < kCodes; ++c) {
                const bool match = code == (uint32_t)c || code == 4u || c == 4;
                T v = (T)0;
                if (real && c != kPad) v = match ? (T)p.lm : -(T)p.lx;
                *slot(c, r) = v;
            }
        }
    }

    // S: forward steps of the pair's group (a multiple of the checkpoint
    // block); hs_bytes: LDS bytes per group for the staged haplotype (it
    // follows the emission table).
    __device__ __forceinline__ void init(const AdjArgs &A, char *lds, const AdjRec &r_in, int S_in, int hs_bytes)
    {
        lane = threadIdx.x;
        g = lane / P;
        t = lane % P;
        rec = r_in;
        S = S_in;
        const DevProblem &pb = A.pb;
        ro = pb.read_offset[rec.read];
        m = (int)(pb.read_offset[rec.read + 1] - ro);
        n = rec.n;
        rml = m - t * K;
        bad = false;
        E = lds;
        char *mine = E + lane * C::ENT;
        if constexpr (HAT) {
            init_rows_hat(A, mine);
        } else {
            init_rows_plain(A, mine);
        }
        // D(0, j) = 1/n times the first read row's beta (it multiplies that
        // D in both forms), scaled
        edge = (t == 0) ? (T)(ldexp(load_beta(pb, A.lin_params, ro, c_prob), AdjRange<T>::kFwd) / (double)n) : (T)0;
        uint8_t *h = (uint8_t *)(lds + C::E_BYTES + g * hs_bytes);
        const uint8_t *hap = pb.hap_bases + pb.hap_offset[rec.hap];
        const int len = S + P + 2;
        // 8 columns per lane in flight at a time: the loads do not wait on
        // each other
        for (int x0 = t; x0 < len; x0 += 8 * P) {
            uint32_t v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int j = x0 + k * P - P;
                v[k] = (j >= 1 && j <= n) ? clamp_code(hap[j - 1]) : (uint32_t)kPad;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (x0 + k * P < len) h[x0 + k * P] = (uint8_t)v[k];
        }
        hs = h;
        El = mine;
        ckl = (T *)(lds + C::E_BYTES + C::G * hs_bytes);
        __syncthreads();
    }

    // the code of the lane's column at step s, and that code's table column
    __device__ __forceinline__ int hcode(int s) const { return hs[s - t + 1 + P]; }
    __device__ __forceinline__ const char *ecol(int s) const { return El + hcode(s) * C::CODE_BYTES; }
};

// Lane t receives lane t-1's value.  With the rescaled states (FP32) a
// 32-lane group's first lane may take the previous group's last row from a
// single wave shift: that row is the absorbing row or past it (Ih exactly
// zero, M and Dh only meeting zero coefficients), so one DPP move serves
// every group size.
template <typename T, int P>
__device__ __forceinline__ T adj_up(T v)
{
    if constexpr (sizeof(T) == 4 && P == 32)
        return __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
    else
        return shift_up<P>(v);
}

// One forward step of the lane's K rows: (mo, io, do_) hold column j-1 on
// entry, (mn, in, dn) receive column j; (mu, iu) and (md, id, dd) are the row
// above at columns j and j-1.  FP32: the rescaled states (M, Ih, Dh); FP64:
// (M, I, D').
template <typename T, int P, int K>
__device__ __forceinline__ void adj_cell_step(const AdjPair<T, P, K> &pr, const T (&mo)[K], const T (&io)[K],
                                              const T (&do_)[K], T (&mn)[K], T (&in)[K], T (&dn)[K], T mu, T iu,
                                              T md, T id, T dd, const T *lam)
{
#pragma unroll
    for (int r = 0; r < K; ++r) {
        T mr, ir, dr;
        if constexpr (AdjPair<T, P, K>::HAT) {
            mr = fabs(lam[r]) * fma(pr.al[r], md, fma(pr.cd[r], dd, id));
            ir = fma(pr.ke[r], iu, pr.kd[r] * mu);
            dr = fma(pr.ep[r], do_[r], mo[r]);
        } else {
            mr = fabs(lam[r]) * fma(pr.al[r], md, fma(pr.be[r], id, dd));
            ir = fma(pr.ep[r], iu, pr.de[r] * mu);
            dr = fma(pr.ep[r], do_[r], pr.ze[r] * mo[r]);
        }
        md = mo[r];
        id = io[r];
        dd = do_[r];
        mn[r] = mr;
        in[r] = ir;
        dn[r] = dr;
        mu = mr;
        iu = ir;
    }
}

// The values a lane receives from the lane above at one step: (M, I, D) of
// its last row, with the first lane's row-0 boundary D added in (through Ih
// with the rescaled states, through D' otherwise).
template <typename T, int P, int K>
__device__ __forceinline__ void adj_from_above(const AdjPair<T, P, K> &pr, const T (&M)[K], const T (&I)[K],
                                               const T (&D)[K], T &mu, T &iu, T &du)
{
    constexpr bool HAT = AdjPair<T, P, K>::HAT;
    mu = adj_up<T, P>(M[K - 1]);
    iu = adj_up<T, P>(I[K - 1]) + (HAT ? pr.edge : (T)0);
    du = adj_up<T, P>(D[K - 1]) + (HAT ? (T)0 : pr.edge);
}

// Checkpointed forward of the wave's pairs.  ck: the workgroup's slice,
// [S/CB][3K+3][64] values (lane state M, I, D and the diagonal md, id, dd
// before steps 0, CB, 2 CB, ...).  Returns the scaled row-m sum, in the lane
// that holds the absorbing row (FP32: its Dh, flushed into FP64 every 64
// steps; nothing reads that Dh, so zeroing it is invisible to the backward)
// or in lane P-1 of each group (FP64: the passed-down I of the last row).
template <typename T, int K>
struct AdjCk {
    static constexpr int V = 3 * K + 3;  // values per lane per checkpoint
};

template <typename T, int P, int K>
__device__ __forceinline__ T adj_take_dm(const AdjPair<T, P, K> &pr, T (&D)[K])
{
    T dm = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        dm = r == pr.rml ? D[r] : dm;
        D[r] = r == pr.rml ? (T)0 : D[r];
    }
    return dm;
}

template <typename T, int P, int K, int CB>
__device__ __forceinline__ double adj_forward(const AdjPair<T, P, K> &pr, T *ck)
{
    constexpr bool HAT = AdjPair<T, P, K>::HAT;
    constexpr int V = AdjCk<T, K>::V;
    const int S = pr.S;
    T M[K], I[K], D[K];
#pragma unroll
    for (int r = 0; r < K; ++r) M[r] = I[r] = D[r] = (T)0;
    T md = 0, id = HAT ? pr.edge : (T)0, dd = HAT ? (T)0 : pr.edge;
    double acc = 0.0;  // row-m sum: partial sums in T over 64 steps, then FP64
    T part = 0;
    for (int s0 = 0; s0 < S; s0 += CB) {
        if ((s0 & 63) == 0) {
            if constexpr (HAT)
                acc += (double)adj_take_dm<T, P, K>(pr, D);
            else
                acc += (double)part;
            part = 0;
        }
        T *cq = ck + (int64_t)(s0 / CB) * V * 64 + pr.lane;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            cq[r * 64] = M[r];
            cq[(K + r) * 64] = I[r];
            cq[(2 * K + r) * 64] = D[r];
        }
        cq[3 * K * 64] = md;
        cq[(3 * K + 1) * 64] = id;
        cq[(3 * K + 2) * 64] = dd;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            T mu, iu, du;
            adj_from_above<T, P, K>(pr, M, I, D, mu, iu, du);
            T lam[K];
            const char *e = pr.ecol(s0 + c);
#pragma unroll
            for (int r = 0; r < K; ++r) lam[r] = *(const T *)(e + r * AdjCfg<T, P, K>::ROW_BYTES);
            adj_cell_step<T, P, K>(pr, M, I, D, M, I, D, mu, iu, md, id, dd, lam);
            md = mu;
            id = iu;
            dd = du;
            if constexpr (!HAT) part += I[K - 1];
        }
    }
    if constexpr (HAT)
        return acc + (double)adj_take_dm<T, P, K>(pr, D);  // the last M of that row is zero
    else
        return acc + (double)part;
}

template <typename T, int K>
__device__ __forceinline__ void adj_load_ck(const T *ck, int q, int lane, T (&cq)[AdjCk<T, K>::V])
{
    constexpr int V = AdjCk<T, K>::V;
    const T *c0 = ck + (int64_t)q * V * 64 + lane;
#pragma unroll
    for (int v = 0; v < V; ++v) cq[v] = c0[v * 64];
}

// FP32: checkpoint q is copied from the workspace into the wave's LDS
// buffer ckl ([V][64], the workspace's own layout) by the memory unit
// (global_load_lds), so a block's checkpoint is in flight during the
// previous block without holding registers.  Completion is tracked by vmcnt.
template <int K>
__device__ __forceinline__ void adj_stage_ck(const float *ck, int q, int lane, float *ckl)
{
    constexpr int V = AdjCk<float, K>::V;
    const float *c0 = ck + (int64_t)q * V * 64 + lane;
#pragma unroll
    for (int v = 0; v < V; ++v)
        __builtin_amdgcn_global_load_lds((const void *)(c0 + v * 64),
                                         (__attribute__((address_space(3))) void *)(ckl + v * 64), 4, 0, 0);
}

// s_waitcnt on gfx9: vmcnt(0) (every vector memory operation of the wave,
// LDS copies included, has completed), lgkmcnt(0) (every LDS read has
// returned); each also a compiler barrier for memory
__device__ __forceinline__ void wait_vm0()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// vmcnt(N) for N < 64: at most N vector memory operations of the wave
// still outstanding
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt has 6 bits");
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(((N >> 4) << 14) | 0x0f70 | (N & 15));
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ void wait_lgkm0()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Eight row sums of forward value x backward value, per row of the lane:
// the alpha and the beta terms of M, each split into match columns (am, bm)
// and mismatch columns (ax, bx, accumulated negative), delta, eps (insert),
// eps (delete), zeta.  Every M(i,j) B_M(i,j) is its alpha term plus its beta
// term, so the emission uses follow as sums of same-signed parts: match
// alpha am + bm, mismatch -(alpha ax + bx); alpha and beta as
// alpha (am - ax) and bm - bx.  No use count is a difference of two sums
// (taking the match uses as alpha + beta - mismatch uses would cancel on
// rows where nearly every probable alignment mismatches).
template <typename T, int K>
struct AdjSums {
    T am[K], ax[K], bm[K], bx[K], d[K], ei[K], ed[K], z[K];
};

// Reverse wavefront over the checkpointed forward of the wave's pairs.
// Checkpoints are R blocks of CB steps apart: fine block f of a checkpoint
// interval is rebuilt by advancing f CB steps from the checkpoint and then
// recomputing its CB steps into registers.
//
// FP32 (rescaled states), with Bl = lam B_M:
//   B_M(i,j)  = al_{i+1} Bl(i+1,j+1) + kd_{i+1} B_Ih(i+1,j) + B_Dh(i,j+1)
//   B_Ih(i,j) =          Bl(i+1,j+1) + ke_{i+1} B_Ih(i+1,j)
//   B_Dh(i,j) = cd_{i+1} Bl(i+1,j+1) + ep_i     B_Dh(i,j+1)
// seeded with B_Dh = bscale on the absorbing row (L is its row sum), which
// that row's unit coefficients carry to every column.  FP64 (M, I, D'): the
// recurrences of the file header, seeded through B_I below the group's last
// lane.
template <typename T, int P, int K, int CB, int R = 1>
__device__ __forceinline__ void adj_backward(const AdjPair<T, P, K> &pr, const T *ck, T bscale, AdjSums<T, K> &A)
{
    constexpr bool HAT = AdjPair<T, P, K>::HAT;
    using C = AdjCfg<T, P, K>;
    using V2 = typename Pair2<T>::V;
    constexpr int V = AdjCk<T, K>::V;
    const int t = pr.t, S = pr.S;
    // coefficients of the row below the lane's last row: the next lane's
    // first row; in the group's last lane the shift brings the next group's
    // (or nothing), and keep = 0 masks it and the B values it sends.  Every
    // lane runs the shifts (a DPP move under a lane mask reads 0 from the
    // lanes the mask turns off).
    const bool last = t == P - 1;
    const T keep = last ? (T)0 : (T)1;
    T an_x, bn_x, dn_x, en_x, cn_x, kn_x;
    if constexpr (HAT) {
        an_x = keep * shift_down_raw<P>(pr.al[0]);
        cn_x = keep * shift_down_raw<P>(pr.cd[0]);
        dn_x = keep * shift_down_raw<P>(pr.kd[0]);
        kn_x = keep * shift_down_raw<P>(pr.ke[0]);
        bn_x = en_x = (T)0;
    } else {
        an_x = keep * shift_down_raw<P>(pr.al[0]);
        bn_x = keep * shift_down_raw<P>(pr.be[0]);
        dn_x = keep * shift_down_raw<P>(pr.de[0]);
        en_x = fma(keep, shift_down_raw<P>(pr.ep[0]), (T)1 - keep);
        cn_x = kn_x = (T)0;
    }
    const T edge_bi = (!HAT && last) ? bscale : (T)0;

    T BI[K], BD[K], BL[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        BI[r] = BL[r] = (T)0;
        BD[r] = (HAT && r == pr.rml) ? bscale : (T)0;
        A.am[r] = A.ax[r] = A.bm[r] = A.bx[r] = A.d[r] = A.ei[r] = A.ed[r] = A.z[r] = (T)0;
    }
    T bl_dn_prev = 0;

    const int NB = S / CB;  // fine blocks; the checkpoint of block b is b / R
    // The checkpoint of the next block is fetched during the current one:
    // FP32 into the wave's LDS buffer (no registers held), FP64 into registers.
    constexpr bool LDSPF = sizeof(T) == 4;
    constexpr bool PREFETCH = !LDSPF && PH_ADJ_PREFETCH;
    T cn[V];
    // FP32: two LDS buffers, checkpoint q in buffer q & 1.  The copy of
    // checkpoint q - 2 starts once the last block of checkpoint q has read
    // its buffer, so every copy has the blocks of a whole checkpoint interval
    // to arrive; at any block at most the copies of q and q - 1 are in
    // flight, and vmcnt(V) (the V loads of the later one may remain) means
    // that q's has landed.
    auto ckbuf = [&](int q) { return (float *)pr.ckl + (q & 1) * V * 64; };
    if constexpr (LDSPF) {
        wait_vm0();  // the forward's checkpoint stores have completed
        const int q0 = (NB - 1) / R;
        adj_stage_ck<K>((const float *)ck, q0, pr.lane, ckbuf(q0));
        if (q0 > 0) adj_stage_ck<K>((const float *)ck, q0 - 1, pr.lane, ckbuf(q0 - 1));
    }
    if constexpr (PREFETCH) adj_load_ck<T, K>(ck, (NB - 1) / R, pr.lane, cn);
    for (int b = NB - 1; b >= 0; --b) {
        if constexpr (LDSPF) {
            const int q = b / R;
            if (q > 0)
                wait_vm<V>();
            else
                wait_vm0();
            const float *cb = ckbuf(q);
#pragma unroll
            for (int v = 0; v < V; ++v) cn[v] = cb[v * 64 + pr.lane];
            if (b == q * R && q >= 2) {
                wait_lgkm0();  // the reads above have the buffer's values before it is refilled
                adj_stage_ck<K>((const float *)ck, q - 2, pr.lane, ckbuf(q - 2));
            }
        } else if constexpr (!PREFETCH) {
            adj_load_ck<T, K>(ck, b / R, pr.lane, cn);
        }
        const int q = b;  // steps of this block: q CB .. q CB + CB - 1
        // F[c]: lane state before step q CB + c; bb[c]: the values received
        // from the lane above at step q CB + c - 1 (bb[0]: from the checkpoint)
        T F[CB + 1][3][K];
        T bb[CB + 1][3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
#pragma unroll
            for (int r = 0; r < K; ++r) F[0][v][r] = cn[v * K + r];
            bb[0][v] = cn[3 * K + v];
        }
        if (PREFETCH && b > 0) adj_load_ck<T, K>(ck, (b - 1) / R, pr.lane, cn);

        if constexpr (R > 1) {
            // advance from the checkpoint at step (b / R) R CB to step q CB,
            // CB steps at a time
#pragma unroll 1
            for (int s0 = (b / R) * R * CB; s0 < q * CB; s0 += CB) {
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    T mu, iu, du;
                    adj_from_above<T, P, K>(pr, F[0][0], F[0][1], F[0][2], mu, iu, du);
                    T lam[K];
                    const char *e = pr.ecol(s0 + c);
#pragma unroll
                    for (int r = 0; r < K; ++r) lam[r] = *(const T *)(e + r * C::ROW_BYTES);
                    adj_cell_step<T, P, K>(pr, F[0][0], F[0][1], F[0][2], F[0][0], F[0][1], F[0][2], mu, iu,
                                           bb[0][0], bb[0][1], bb[0][2], lam);
                    bb[0][0] = mu;
                    bb[0][1] = iu;
                    bb[0][2] = du;
                }
            }
        }

        // recompute the block as a wavefront
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            adj_from_above<T, P, K>(pr, F[c][0], F[c][1], F[c][2], bb[c + 1][0], bb[c + 1][1], bb[c + 1][2]);
            T lam[K];
            const char *e = pr.ecol(q * CB + c);
#pragma unroll
            for (int r = 0; r < K; ++r) lam[r] = *(const T *)(e + r * C::ROW_BYTES);
            adj_cell_step<T, P, K>(pr, F[c][0], F[c][1], F[c][2], F[c + 1][0], F[c + 1][1], F[c + 1][2],
                                   bb[c + 1][0], bb[c + 1][1], bb[c][0], bb[c][1], bb[c][2], lam);
        }

        // reverse wavefront over the block
#pragma unroll
        for (int c = CB - 1; c >= 0; --c) {
            const int code = pr.hcode(q * CB + c);
            const char *e = pr.El + code * C::CODE_BYTES;
            T lam[K];
#pragma unroll
            for (int r = 0; r < K; ++r) lam[r] = *(const T *)(e + r * C::ROW_BYTES);
            const T bi_dn = fma(keep, shift_down_raw<P>(BI[0]), edge_bi);
            const T bl_dn = keep * shift_down_raw<P>(BL[0]);  // Bl of the row below, next column
            T bid = bi_dn;            // B_I of the row below, this column
            T bl_below = bl_dn_prev;  // Bl of the row below, next column
#pragma unroll
            for (int r = K - 1; r >= 0; --r) {
                const T bld = fabs(bl_below);  // BL carries the table entry's sign
                // forward values around (i, j): row above at j and j-1, own row at j-1 and j
                const T mu = (r == 0) ? bb[c + 1][0] : F[c + 1][0][r - 1];
                const T iu = (r == 0) ? bb[c + 1][1] : F[c + 1][1][r - 1];
                const T mdg = (r == 0) ? bb[c][0] : F[c][0][r - 1];
                const T idg = (r == 0) ? bb[c][1] : F[c][1][r - 1];
                const T ddg = (r == 0) ? bb[c][2] : F[c][2][r - 1];
                T bi, bd, bm;
                if constexpr (HAT) {
                    const T an = (r == K - 1) ? an_x : pr.al[r + 1];
                    const T cn_ = (r == K - 1) ? cn_x : pr.cd[r + 1];
                    const T dn = (r == K - 1) ? dn_x : pr.kd[r + 1];
                    const T kn = (r == K - 1) ? kn_x : pr.ke[r + 1];
                    bi = fma(kn, bid, bld);
                    bd = fma(pr.ep[r], BD[r], cn_ * bld);
                    bm = fma(an, bld, fma(dn, bid, BD[r]));
                } else {
                    const T an = (r == K - 1) ? an_x : pr.al[r + 1];
                    const T bnr = (r == K - 1) ? bn_x : pr.be[r + 1];
                    const T dn = (r == K - 1) ? dn_x : pr.de[r + 1];
                    const T en = (r == K - 1) ? en_x : pr.ep[r + 1];
                    bi = fma(en, bid, bnr * bld);
                    bd = fma(pr.ep[r], BD[r], bld);  // B_D' = Bl below-right + eps B_D' right
                    bm = fma(an, bld, fma(dn, bid, pr.ze[r] * BD[r]));
                }
                // Bl with the sign of the table entry: negative on a mismatch
                // column; its match and mismatch parts (the other part is 0)
                const T bl = lam[r] * bm;
                const T blm = fmax(bl, (T)0), blx = fmin(bl, (T)0);
                A.am[r] = fma(mdg, blm, A.am[r]);
                A.ax[r] = fma(mdg, blx, A.ax[r]);
                T y;  // the beta term's forward factor
                if constexpr (HAT)
                    y = fma(pr.cd[r], ddg, idg);  // (Ih + cD Dh)_diag
                else
                    y = fma(pr.be[r], idg, ddg);  // (beta I + D')_diag
                A.bm[r] = fma(y, blm, A.bm[r]);
                A.bx[r] = fma(y, blx, A.bx[r]);
                A.d[r] = fma(mu, bi, A.d[r]);
                A.ei[r] = fma(iu, bi, A.ei[r]);
                A.ed[r] = fma(F[c][2][r], bd, A.ed[r]);
                A.z[r] = fma(F[c][0][r], bd, A.z[r]);
                bl_below = BL[r];  // still the next column's value: row r-1's diagonal
                BI[r] = bi;
                BD[r] = bd;
                BL[r] = bl;
                bid = bi;
            }
            bl_dn_prev = bl_dn;
        }
    }
}

// Destination of row i of the pair's gradient: the read's own row when the
// read has no other pair, else the pair's row of the per-pair array.
template <typename T, int P, int K>
__device__ __forceinline__ float *adj_row(const AdjArgs &A, const AdjPair<T, P, K> &pr, int i)
{
    return pr.rec.direct ? A.grad_out + (pr.ro + i) * 7 : A.grad_pair + (pr.rec.grow + i) * 7;
}

// Expected uses per row, g = coefficient x sum / (L_s 2^SB), times the
// pair's upstream gradient u, stored (plain stores: every row has one
// writer) at the pair's rows.  The coefficient is the one the sum's backward
// value multiplies in the DP: FP32 alpha, kD (delta's), kE and eps (eps's
// two terms), 1 (zeta's: M -> Dh has a unit coefficient); FP64 alpha,
// delta, eps, zeta'.  beta's sum already holds beta.
template <typename T, int P, int K>
__device__ __forceinline__ void adj_emit(const AdjArgs &A, const AdjPair<T, P, K> &pr, double u, double inv,
                                         const AdjSums<T, K> &s)
{
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = pr.t * K + r;
        if (i >= pr.m) continue;
        const double al = (double)pr.al[r];
        const double am = (double)s.am[r], ax = (double)s.ax[r], bm = (double)s.bm[r], bx = (double)s.bx[r];
        const double ga = al * (am - ax) * inv;    // ax <= 0, bx <= 0
        const double gb = (bm - bx) * inv;
        const double gx = -(al * ax + bx) * inv;  // mismatch emissions
        const double gm = (al * am + bm) * inv;   // match emissions
        double gd, ge, gz;
        if constexpr (AdjPair<T, P, K>::HAT) {
            gd = (double)pr.kd[r] * (double)s.d[r] * inv;
            ge = ((double)pr.ke[r] * (double)s.ei[r] + (double)pr.ep[r] * (double)s.ed[r]) * inv;
            gz = (double)s.z[r] * inv;
        } else {
            gd = (double)pr.de[r] * (double)s.d[r] * inv;
            ge = (double)pr.ep[r] * ((double)s.ei[r] + (double)s.ed[r]) * inv;
            gz = (double)pr.ze[r] * (double)s.z[r] * inv;
        }
        float *o = adj_row<T, P, K>(A, pr, i);
        o[0] = (float)(u * ga);
        o[1] = (float)(u * gb);
        o[2] = (float)(u * gd);
        o[3] = (float)(u * ge);
        o[4] = (float)(u * gz);
        o[5] = (float)(u * gm);
        o[6] = (float)(u * gx);
    }
}

// A pair with upstream gradient 0 contributes zeros (whatever its range).
template <typename T, int P, int K>
__device__ __forceinline__ void adj_emit_zero(const AdjArgs &A, const AdjPair<T, P, K> &pr)
{
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const int i = pr.t * K + r;
        if (i >= pr.m) continue;
        float *o = adj_row<T, P, K>(A, pr, i);
#pragma unroll
        for (int c = 0; c < 7; ++c) o[c] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// FP32 pass: a persistent grid drains the tiles of one (P, K) configuration.
// Groups past the end of the record list mirror group 0 and emit nothing.
// ---------------------------------------------------------------------------
#ifndef PH_ADJ_WAVES
#define PH_ADJ_WAVES 2
#endif
template <int P, int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K <= 3 ? 3 : PH_ADJ_WAVES))) void k_adj32(AdjArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int G = 64 / P;
    const int g = (int)threadIdx.x / P;
    float *ck = A.ws + (int64_t)blockIdx.x * A.ws_stride;
    for (int tile = next_tile(A.tile_next); tile < A.ntiles; tile = next_tile(A.tile_next)) {
        const int first = tile * G, idx = first + g;
        const bool valid = idx < A.nrec;
        const AdjRec rec = A.recs[valid ? idx : first];
        AdjPair<float, P, K> pr;
        pr.init(A, lds, rec, __builtin_amdgcn_readlane(rec.S, 0), A.hs_bytes);
        const double acc = adj_forward<float, P, K, kAdjC * kAdjR>(pr, ck);
        // the absorbing row's lane holds the sum; a group with a beta below
        // 2^-20 goes to the FP64 pass like a pair outside the FP32 range
        const double Ls = __shfl(acc, g * P + min(pr.m / K, P - 1));
        const uint64_t badm = __ballot(pr.bad);
        const uint64_t gm = P == 64 ? ~0ull : (((1ull << P) - 1) << (g * P));
        const bool good = (badm & gm) == 0 && (Ls >= A.threshold) && (Ls <= 3.0e38);
        const int SB = good ? AdjRange<float>::kProd - ilogb(Ls) : 0;
        AdjSums<float, K> sums;
        adj_backward<float, P, K, kAdjC, kAdjR>(pr, ck, good ? ldexpf(1.f, SB) : 0.f, sums);
        const double u = valid ? A.grad_in[rec.out] : 0.0;
        if (!valid) {
            // a group past the end of the records mirrors group 0: no output
        } else if (u == 0.0) {  // a pair with u = 0 contributes nothing, whatever its range
            adj_emit_zero<float, P, K>(A, pr);
        } else {
            if (good) {
                adj_emit<float, P, K>(A, pr, u, 1.0 / ldexp(Ls, SB), sums);
            } else if (pr.t == 0) {
                // outside the FP32 range: queued for the FP64 pass, class
                // K64 - 1 with K64 = ceil((m + 1) / 64) rows per lane
                const int cls = (pr.m + 64) / 64 - 1;
                const int slot = atomicAdd(&A.q64_count[cls], 1);
                A.q64[(int64_t)cls * A.q64_stride + slot] = (int32_t)(A.rec_base + idx);
            }
        }
        __syncthreads();  // LDS tables are rebuilt for the next tile
    }
}

// ---------------------------------------------------------------------------
// FP64 pass: a persistent grid drains the queue of class K (64 lanes x K
// rows, reads of 64 (K-1) .. 64 K - 1 bases), one pair at a time per
// workgroup.  Every wave leaves the loop once the cursor passes the queue
// length, which the FP32 pass has finished writing before this launch.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(64) void k_adj64(AdjArgs A)
{
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int P = 64;
    const int cls = K - 1;
    const int count = A.q64_count[cls];
    double *ck = A.ws64 + (int64_t)blockIdx.x * A.ws64_stride;
    for (int item = next_tile(&A.q64_next[cls]); item < count; item = next_tile(&A.q64_next[cls])) {
        const int32_t gi = A.q64[(int64_t)cls * A.q64_stride + item];
        const AdjRec rec = A.all_recs[gi];
        const int S = ((rec.n + P - 1 + kAdjC64 - 1) / kAdjC64) * kAdjC64;
        AdjPair<double, P, K> pr;
        pr.init(A, lds, rec, S, A.hs_bytes64);
        const double acc = adj_forward<double, P, K, kAdjC64>(pr, ck);
        const double Ls = __shfl(acc, P - 1);
        // below the FP64 range floor the pair's gradients are NaN
        const bool good = (Ls >= A.floor64) && isfinite(Ls);
        const int SB = good ? AdjRange<double>::kProd - ilogb(Ls) : 0;
        AdjSums<double, K> sums;
        adj_backward<double, P, K, kAdjC64>(pr, ck, good ? ldexp(1.0, SB) : 0.0, sums);
        adj_emit<double, P, K>(A, pr, A.grad_in[rec.out], good ? 1.0 / ldexp(Ls, SB) : (double)NAN, sums);
        __syncthreads();  // LDS tables are rebuilt for the next pair
    }
}

// Fixed-order sum over the pairs of each read with several pairs:
// grad_out[ro + i][c] = sum over h = 0 .. H-1 of grad_pair[grow + h m + i][c],
// accumulated in FP64 in haplotype order, so the result does not depend on
// which pair finished first.  One workgroup per read.
__global__ __launch_bounds__(256) void k_adj_reduce(const AdjRedRead *reads, const float *gp, float *go)
{
    const AdjRedRead rd = reads[blockIdx.x];
    const int64_t n = (int64_t)rd.m * 7;
    const float *src = gp + rd.grow * 7;
    float *dst = go + rd.ro * 7;
    for (int64_t e = threadIdx.x; e < n; e += 256) {
        double s = 0.0;
        for (int h = 0; h < rd.H; ++h) s += (double)src[(int64_t)h * n + e];
        dst[e] = (float)s;
    }
}

hipError_t launch_adj_reduce(const AdjRedRead *reads, int32_t nreads, const float *grad_pair, float *grad_out,
                             hipStream_t s)
{
    if (nreads <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_reduce, dim3(nreads), dim3(256), 0, s, reads, grad_pair, grad_out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_f32(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.f;
}

__global__ __launch_bounds__(64) void k_zero_i32(int32_t *p, int n)
{
    for (int i = threadIdx.x; i < n; i += 64) p[i] = 0;
}

#define PH_ADJ_CONFIGS(X) X(32, 1) X(32, 2) X(32, 3) X(32, 4) X(32, 5) X(64, 3) X(64, 4) X(64, 5)

bool adj_supported(int P, int K)
{
#define PH_AS(p, k) if (P == p && K == k) return true;
    PH_ADJ_CONFIGS(PH_AS)
#undef PH_AS
    return false;
}

int adj_e_bytes(int P, int K)
{
    (void)P;  // the table holds all 64 lanes of the wave whatever the group size
    return kCodes * K * AdjCfg<float, 64, 1>::ROW_BYTES;
}

int adj64_e_bytes(int K) { return kCodes * K * AdjCfg<double, 64, 1>::ROW_BYTES; }

int adj_ck_lds_bytes(int K) { return 2 * (3 * K + 3) * 64 * (int)sizeof(float); }

static int occupancy(const void *fn, size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, lds) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

hipError_t launch_adj32(const AdjArgs &a, int P, int K, int grid, hipStream_t s)
{
    const size_t lds = (size_t)adj_e_bytes(P, K) + (size_t)(64 / P) * a.hs_bytes + (size_t)adj_ck_lds_bytes(K);
#define PH_LA(p, k)                                                              \
    if (P == p && K == k) {                                                      \
        hipLaunchKernelGGL((k_adj32<p, k>), dim3(grid), dim3(64), lds, s, a);   \
        return hipGetLastError();                                                \
    }
    PH_ADJ_CONFIGS(PH_LA)
#undef PH_LA
    return hipErrorInvalidValue;
}

// resident workgroups per CU, from registers (LDS is small next to 160 KB)
int adj32_blocks_per_cu(int P, int K)
{
#define PH_AO(p, k) if (P == p && K == k) return occupancy((const void *)k_adj32<p, k>, 0);
    PH_ADJ_CONFIGS(PH_AO)
#undef PH_AO
    return 1;
}

int adj64_blocks_per_cu(int K)
{
    switch (K) {
    case 1: return occupancy((const void *)k_adj64<1>, 0);
    case 2: return occupancy((const void *)k_adj64<2>, 0);
    case 3: return occupancy((const void *)k_adj64<3>, 0);
    case 4: return occupancy((const void *)k_adj64<4>, 0);
    case 5: return occupancy((const void *)k_adj64<5>, 0);
    }
    return 1;
}

hipError_t launch_adj64(const AdjArgs &a, int K, int grid, hipStream_t s)
{
    const size_t lds = (size_t)adj64_e_bytes(K) + (size_t)a.hs_bytes64;
    switch (K) {
    case 1: hipLaunchKernelGGL(k_adj64<1>, dim3(grid), dim3(64), lds, s, a); break;
    case 2: hipLaunchKernelGGL(k_adj64<2>, dim3(grid), dim3(64), lds, s, a); break;
    case 3: hipLaunchKernelGGL(k_adj64<3>, dim3(grid), dim3(64), lds, s, a); break;
    case 4: hipLaunchKernelGGL(k_adj64<4>, dim3(grid), dim3(64), lds, s, a); break;
    case 5: hipLaunchKernelGGL(k_adj64<5>, dim3(grid), dim3(64), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s)
{
    int64_t g = (n + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_zero_f32, dim3((int)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace ph
